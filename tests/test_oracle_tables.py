"""Pins of the oracle's periodic plane-wave tables (CPU only).

The strongest pin is Sec. VI.C: the self-mobility of the periodic algorithm, which is set by
the level split, P_F, the k-cube weights and the quasi-continuous shell, must follow the
finite-box law Tr O^P(0) = Tr O^inf(0) (1 - 2.837 a/L) (Eq. "1/L dependence"), a = lambda_min /
lambda_a. Hasimoto's constant to more digits is 2.837297.
"""
import numpy as np
import pytest
from scipy import integrate

from tests.test_oracle_pins import phit_closed, phit_ref

XI = 2.837297  # Hasimoto (1959); the paper prints 2.837


def free_system(O, L, lmax, N=8, lmin=1.0, A0=0.5):
    pos = np.random.default_rng(0).uniform(0, L, (N, 3))
    p = dict(periodic=1, plane_waves=1, box_L=L, lambda_min=lmin, lambda_max=lmax, bond_type="none",
             wca=0, A0=A0, seed=3)
    return O.Oracle(p, [0, N], np.arange(N + 1), pos)


def quad_tail(fun, a, top=3000.0):
    edges = np.concatenate([[a], np.arange(np.ceil(a / np.pi + 1e-9) * np.pi, top, np.pi)])
    return sum(integrate.quad(fun, x0, x1, epsabs=0, epsrel=1e-12)[0] for x0, x1 in zip(edges[:-1], edges[1:])), edges[-1]


def phi2(q):
    return (phit_closed(q) if q > 0.5 else phit_ref(q)) ** 2


def int_I(xs):
    """int_xs^inf I(x) dx = -xs I(xs) + int_xs^inf t^4 phi~^2 dt (integration by parts)."""
    v4, top = quad_tail(lambda t: t ** 4 * phi2(t), xs)
    v4 += 8 * np.pi ** 2 / (3 * top ** 3)
    v3, top = quad_tail(lambda t: t ** 3 * phi2(t), xs)
    v3 += 2 * np.pi ** 2 * top ** -4
    return -xs * v3 + v4


@pytest.mark.parametrize("L,frac", [(16.0, 4), (32.0, 4), (64.0, 4), (16.0, 2), (48.0, 2)])
def test_self_mobility_follows_hasimoto(oracle_mod, L, frac):
    lmin, lmax, A0, N = 1.0, L / frac, 1.0, 1.0
    o = free_system(oracle_mod, L, lmax, lmin=lmin)
    info = o.system_info()
    w = o.cube_weights()
    NL = 15
    rng = np.arange(-NL, NL + 1)
    lx, ly, lz = np.meshgrid(rng, rng, rng, indexing="ij")
    l2 = (lx ** 2 + ly ** 2 + lz ** 2).ravel()
    ks = 2 * np.pi / L
    k2 = ks ** 2 * l2
    nz = l2 > 0
    corner = l2 > (NL + 0.5) ** 2
    # outside-cube modes: continuum beyond k_s minus the cube's corner modes
    xs = ks * (NL + 0.5) * lmax
    shell = (L / (2 * np.pi)) ** 3 * 4 * np.pi * int_I(xs) / lmax - np.sum(w[corner] / k2[corner])
    Nk = info["N_k"]
    dr2_F = Nk * (2 * A0 ** 2 / (5 * N)) * (np.sum(w[nz] / k2[nz]) + shell)
    M3 = 2 * np.pi ** 2 / 105 * (9 - 8 * np.log(2))
    M4 = 8 * np.pi ** 3 / 105
    Nlam = 3 / (lmin ** -3 - lmax ** -3)
    dr2_w = 2 * A0 ** 2 * M4 * Nlam * (1 / lmin - 1 / lmax) / ((2 * np.pi) ** 3 * N)   # Eq. "wavelet dr2"
    dr2_inf = 6 * A0 ** 2 * M4 * lmin ** 2 / ((2 * np.pi) ** 3 * N)                    # lambda_max -> inf
    PF = info["P_F"]
    ratio = ((1 - PF) * dr2_w + PF * dr2_F) / dr2_inf
    a = lmin / (2 / np.pi * M4 / M3)
    assert ratio == pytest.approx(1 - XI * a / L, abs=4e-6)
    # the printed constant, to its printed precision
    assert abs((1 - ratio) * L / a - 2.837) < 0.0006


def test_normalisation_pieces(oracle_mod):
    o = free_system(oracle_mod, 24.0, 6.0)
    info = o.system_info()
    w = o.cube_weights()
    Wtot = info["W_cube"] + info["W_cont"] - info["W_corner"]
    assert info["N_k"] == pytest.approx(1 / Wtot, rel=1e-14)
    assert info["W_cube"] == pytest.approx(np.sum(w), rel=1e-12)
    # P(k=0) = I(0) N_k with I(0) = M3 (Eq. "Prob of k_l")
    assert info["P_k0"] == pytest.approx(oracle_mod.moment(3) * info["N_k"], rel=1e-12)
    # continuum piece: (L/2pi)^3 int_{|k|>k_s} I(k lmax) d^3k by scipy
    L, lmax, ks = 24.0, 6.0, 2 * np.pi / 24.0
    xs = ks * 15.5 * lmax
    v, top = quad_tail(lambda x: x * x * float(oracle_mod.I(x)), xs, top=600.0)
    v += 2 * np.pi ** 2 / top  # x^2 I(x) ~ 2 pi^2 / x^2
    ref = (L / (2 * np.pi)) ** 3 * 4 * np.pi / lmax ** 3 * v
    assert info["W_cont"] == pytest.approx(ref, rel=2e-6)
    # P_F from Eq. "P(Fourier)" with R of the paper's R formula
    R = (L / lmax) ** 3 * oracle_mod.moment(6) * info["N_k"] / (6 * np.pi ** 2)
    assert info["R"] == pytest.approx(R, rel=1e-13)
    assert info["P_F"] == pytest.approx(1 / (1 + R * ((lmax / 1.0) ** 3 - 1)), rel=1e-13)


@pytest.mark.parametrize("ratio", [4.0, 8.0])
def test_R_tends_to_one(oracle_mod, ratio):
    """For L/lambda_max large the lattice sum becomes the infinite-system integral and R -> 1
    (Sec. V.C: R would be exactly 1 for the infinite system, Eq. "R^inf definition")."""
    o = free_system(oracle_mod, 16.0 * ratio, 16.0)
    assert abs(o.system_info()["R"] - 1) < 2e-4


def test_shell_inverse_table(oracle_mod):
    o = free_system(oracle_mod, 32.0, 8.0)
    s = o.shell_table()
    M = len(s) - 1
    assert s[0] == 1.0 and s[-1] == 0.0 and np.all(np.diff(s) < 0)
    xs = 2 * np.pi / 32.0 * 15.5 * 8.0

    def G(x):
        v, top = quad_tail(lambda t: t * t * float(oracle_mod.I(t)), x, top=max(4 * x, 600.0))
        return v + 2 * np.pi ** 2 / top

    G0 = G(xs)
    for i in (512, 2048, 3500):
        assert G(xs / s[i]) == pytest.approx((1 - i / M) * G0, rel=1e-6)
