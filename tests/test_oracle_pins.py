"""Pins of the oracle's building blocks against the paper and the mathematics (CPU only).

Each check uses something other than the oracle's own formula: published known-answer
vectors, scipy quadrature of the paper's definitions, finite differences, or exact algebra.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, stats

M_PI = math.pi


def phit_ref(q):
    """phi~(q) by direct quadrature of the radial transform of phi(r) = r^2/2 - r^3/3 - 1/6
    (Eq. "Scalar wavelet position"), independent of the closed form and of any series."""
    f = lambda r: r * r * (r * r / 2 - r ** 3 / 3 - 1 / 6) * (np.sinc(q * r / np.pi))
    return 4 * np.pi * integrate.quad(f, 0.0, 1.0, epsabs=0, epsrel=1e-13, limit=200)[0]


def phit_closed(q):
    """Eq. "Scalar wavelet Fourier" as printed."""
    return 4 * np.pi * q ** -6 * (5 * q * np.sin(q) - (q * q - 8) * np.cos(q) - 8)


# ---------------------------------------------------------------------------- Philox
def test_philox_known_answers(oracle_mod, golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle_mod.philox(v[0:4], v[4:6]) == v[6:10]


def test_stream_uniform_and_distinct(oracle_mod):
    # one sub-stream holds 8192 doubles (12-bit block index); pool 25 sub-streams
    co = np.concatenate([oracle_mod.stream_doubles(12345, 3, 7, 2, 55, t, 0, 0, 8192)[0] for t in range(25)])
    _, oc = oracle_mod.stream_doubles(12345, 3, 7, 2, 55, 0, 0, 0, 8192)
    assert co.min() >= 0.0 and co.max() < 1.0
    assert oc.min() > 0.0 and oc.max() <= 1.0
    np.testing.assert_array_equal(oc - co[:8192], np.full(8192, 2.0 ** -53))
    assert len(np.unique(co)) == len(co)
    # chi-square uniformity over 64 bins
    h, _ = np.histogram(co, bins=64, range=(0, 1))
    assert stats.chisquare(h).pvalue > 1e-4
    # neighbouring counters give unrelated streams
    co2, _ = oracle_mod.stream_doubles(12345, 3, 7, 2, 56, 0, 0, 0, 8192)
    assert abs(np.corrcoef(co[:8192], co2)[0, 1]) < 0.05
    # retry and try indices address distinct streams too
    co3, _ = oracle_mod.stream_doubles(12345, 3, 7, 2, 55, 9, 1, 0, 16)
    co4, _ = oracle_mod.stream_doubles(12345, 3, 7, 2, 55, 9, 0, 1, 16)
    assert not np.array_equal(co[:16], co3) and not np.array_equal(co3, co4)


# ------------------------------------------------------------------ wavelet transform
@pytest.mark.parametrize("q", [1e-3, 0.1, 0.7, 1.9, 2.999, 3.0, 4.5, 10.0, 33.3])
def test_phit_matches_radial_transform(oracle_mod, q):
    ref = phit_ref(q)
    assert oracle_mod.phit(q) == pytest.approx(ref, rel=1e-11, abs=1e-15)
    if q > 0.5:
        assert phit_closed(q) == pytest.approx(ref, rel=1e-9)


def test_phit_at_zero_is_volume_integral(oracle_mod):
    # phi~(0) = int phi d^3r = 4 pi (1/10 - 1/18 - 1/18) = -2 pi / 45
    assert oracle_mod.phit(0.0) == pytest.approx(-2 * np.pi / 45, rel=1e-15)


def moment_quad(m):
    f = lambda k: k ** m * phit_closed(k) ** 2 if k > 0.5 else k ** m * phit_ref(k) ** 2
    edges = np.concatenate([[0.0, 0.5], np.arange(np.pi, 4000.0, np.pi)])
    val = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-12)[0] for a, b in zip(edges[:-1], edges[1:]))
    # tail beyond the last edge from the asymptote k^m phi~^2 ~ 16 pi^2 k^(m-8) cos^2 k
    return val + 8 * np.pi ** 2 * edges[-1] ** (m - 7) / (7 - m)


def test_moments_closed_forms(oracle_mod):
    """M3 = (2 pi^2/105)(9 - 8 ln 2), M4 = 8 pi^3/105, M6 = 8 pi^3/5 (Eq. "phi moment")."""
    assert oracle_mod.moment(3) == pytest.approx(moment_quad(3), rel=1e-9)
    assert oracle_mod.moment(4) == pytest.approx(moment_quad(4), rel=1e-8)
    assert oracle_mod.moment(6) == pytest.approx(moment_quad(6), rel=1e-6)


def test_lambda_a_matches_paper(oracle_mod, golden_dir):
    """lambda_a = (2/pi) M4/M3 = ((9/8) - ln 2)^-1 ~ 2.316 (Eq. "lambda_a")."""
    lam_a = 2 / np.pi * oracle_mod.moment(4) / oracle_mod.moment(3)
    assert lam_a == pytest.approx(1.0 / (9.0 / 8.0 - np.log(2.0)), rel=1e-14)
    printed = {l.split()[0]: l.split()[1:3] for l in open(os.path.join(golden_dir, "paper_constants.txt"))
               if l.strip() and not l.startswith("#")}
    v, tol = map(float, printed["lambda_a"])
    assert abs(lam_a - v) <= tol


@pytest.mark.parametrize("x", [0.0, 0.3, 1.0, 2.5, 7.0, 15.3, 40.0, 81.0])
def test_I_matches_quadrature(oracle_mod, x):
    f = lambda q: q ** 3 * (phit_closed(q) if q > 0.5 else phit_ref(q)) ** 2
    edges = np.concatenate([[x], np.arange(np.ceil(x / np.pi + 1e-9) * np.pi, 3000.0, np.pi)])
    ref = sum(integrate.quad(f, a, b, epsabs=0, epsrel=1e-12)[0] for a, b in zip(edges[:-1], edges[1:]))
    ref += 2 * np.pi ** 2 * edges[-1] ** -4
    assert oracle_mod.I(x) == pytest.approx(ref, rel=1e-8)
    if x == 0.0:
        assert oracle_mod.I(0.0) == pytest.approx(oracle_mod.moment(3), rel=1e-13)


def test_J6_limits(oracle_mod):
    assert oracle_mod.J6(0.0) == pytest.approx(oracle_mod.moment(6), rel=1e-10)
    # far tail: J6 ~ 8 pi^2 / x
    assert oracle_mod.J6(5000.0) == pytest.approx(8 * np.pi ** 2 / 5000.0, rel=1e-3)


def test_time_step_constant():
    """dt w+F = 6 A0^2 M4 lambda_a^2 / ((2 pi)^3 N) = (2/35) lambda_a^2 A0^2 / N (Eq. "dt w+F")."""
    M3 = 2 * np.pi ** 2 / 105 * (9 - 8 * np.log(2))
    M4 = 8 * np.pi ** 3 / 105
    lam_a = 2 / np.pi * M4 / M3
    c = 6 * M4 * lam_a ** 2 / (2 * np.pi) ** 3
    assert c == pytest.approx(2.0 / 35.0 * lam_a ** 2, rel=1e-14)
    assert c == pytest.approx(0.306401, abs=5e-7)


# ------------------------------------------------------------------ lambda sampling
def test_inv_cbrt_exact_to_an_ulp(oracle_mod):
    xs = np.concatenate([np.linspace(0.125, 1.0, 4001), [0.125, 1.0, 0.5, 0.3333333333333333]])
    for x in xs:
        ref = x ** (-1.0 / 3.0)
        got = oracle_mod.inv_cbrt(float(x))
        assert abs(got - ref) <= 2 * np.spacing(ref)


def test_lambda_band_distribution(oracle_mod):
    """lambda on [lo, hi) has PDF ~ lambda^-4 (Eq. "PDF for lambda"); KS test of the inverse
    transform of App. D with band edges."""
    lo, hi = 1.0, 2.0
    co = np.concatenate([oracle_mod.stream_doubles(99, 0, 0, 0, 0, t, 0, 0, 8192)[0] for t in range(5)])
    lam = np.array([oracle_mod.draw_lambda(u, lo, hi) for u in co])
    assert lam.min() >= lo and lam.max() < hi * (1 + 1e-15)
    cdf = lambda x: (lo ** -3 - np.asarray(x) ** -3) / (lo ** -3 - hi ** -3)
    assert stats.kstest(lam, cdf).pvalue > 1e-3
    # the endpoints of the map
    assert oracle_mod.draw_lambda(0.0, lo, hi) == lo


# ------------------------------------------------------------------ the vector wavelet
def test_wavelet_field_properties(oracle_mod):
    rng = np.random.default_rng(5)
    for _ in range(50):
        p = rng.normal(size=3)
        p /= np.linalg.norm(p)
        x = rng.uniform(-0.7, 0.7, size=3)
        w = oracle_mod.wavelet(x, p)
        # transverse to x and to p, antisymmetric in p
        assert abs(w @ x) < 1e-14 and abs(w @ p) < 1e-14
        np.testing.assert_allclose(oracle_mod.wavelet(x, -p), -w, atol=1e-15)
        # divergence free (Eq. "wavelet divergencelessness") by central differences
        if np.linalg.norm(x) < 0.95:
            h = 1e-5
            div = 0.0
            for a in range(3):
                e = np.zeros(3)
                e[a] = h
                div += (oracle_mod.wavelet(x + e, p)[a] - oracle_mod.wavelet(x - e, p)[a]) / (2 * h)
            assert abs(div) < 1e-8
    # zero on and outside the unit sphere (Eq. "wavelet finite extent")
    p = np.array([0.0, 0.0, 1.0])
    assert np.all(oracle_mod.wavelet(np.array([1.0, 0.0, 0.0]), p) == 0)
    assert np.all(oracle_mod.wavelet(np.array([0.0, 1.3, 0.0]), p) == 0)
    # magnitude r sin(theta)(1 - r) (Eq. "Tapered wavelet"): max 1/4 at r = 1/2 in the equator
    np.testing.assert_allclose(np.linalg.norm(oracle_mod.wavelet(np.array([0.5, 0.0, 0.0]), p)), 0.25, rtol=1e-15)
    np.testing.assert_allclose(oracle_mod.wavelet(np.array([0.3, 0.0, 0.4]), p), [0.0, 0.3 * 0.5, 0.0], atol=1e-15)


# ------------------------------------------------------------------ potentials
def test_potentials(oracle_mod):
    """FENE and WCA of Eqs. "FENE potential", "WCA potential"."""
    k, R0 = 30.0, 1.5
    assert oracle_mod.u_fene(R0 * R0 / 2, k, R0) == pytest.approx(-0.5 * k * R0 * R0 * np.log(0.5), rel=1e-15)
    assert math.isinf(oracle_mod.u_fene(R0 * R0, k, R0))
    assert oracle_mod.u_wca(1.0, 1.0, 1.0) == pytest.approx(1.0, rel=1e-15)
    assert oracle_mod.u_wca(2 ** (1 / 3) * 1.000001, 1.0, 1.0) == 0.0
    assert oracle_mod.u_wca(2 ** (1 / 3) * 0.9999999, 1.0, 1.0) == pytest.approx(0.0, abs=1e-5)
    assert math.isinf(oracle_mod.u_wca(0.0, 1.0, 1.0))
