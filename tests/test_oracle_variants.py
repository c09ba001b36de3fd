"""Pins of the oracle's variants against the paper's closed forms (CPU only).

- infinite-system plane waves (Sec. V "Distributions of wavevectors", "The probability of making
  a Fourier move", App. D "Choosing k for an infinite system"):
    * the tabulated inverse of P(k) = N_k k^2 I(k lambda_max), N_k = 3 lambda_max^3 / M6
      (Eqs. "PDF of k", "k normalisation infinite"), against scipy quadrature of phi~;
    * the |k| histogram of the plane waves a sweep makes;
    * with P_F = (lambda_min/lambda_max)^3 (Eq. "P(Fourier) infinite") the plane waves stand in
      exactly for the wavelets above lambda_max (Eq. "R^inf definition"): the relative motion of
      two tracers follows O_w(r; lambda_min, infinity), and free particles diffuse with
      D0 = a^2 / (6 tau) whatever lambda_max is (Eqs. "Oseen (min,infty)", "dt w+F");
- Glauber acceptance (Sec. IV "Choosing the wavelet amplitude", last paragraph): accepted
  fraction 1/(1 + exp(dU/kT)) per dU bin;
- uniform centring (Sec. IV "Distribution of wavelet radii", last paragraph): the same
  two-tracer correlations as the anchored centres, because P_b A_w^2 is the same.
Detailed balance of each variant is pinned in tests/test_oracle_balance.py.
"""
import numpy as np
import pytest
from scipy import integrate

from tests.test_oracle_dynamics import Ow_components
from tests.test_oracle_pins import phit_closed, phit_ref

M3 = 2 * np.pi ** 2 / 105 * (9 - 8 * np.log(2))
M4 = 8 * np.pi ** 3 / 105
M6 = 8 * np.pi ** 3 / 5
LAM_A = 2 / np.pi * M4 / M3


def phi2(q):
    return (phit_closed(q) if q > 0.5 else phit_ref(q)) ** 2


def I_ref(x):
    """I(x) = int_x^inf q^3 phi~(q)^2 dq by scipy, independent of the oracle's quadrature."""
    edges = np.concatenate([[x], np.arange(np.ceil(x / np.pi + 1e-9) * np.pi, 600.0, np.pi)])
    v = sum(integrate.quad(lambda q: q ** 3 * phi2(q), a, b, epsabs=0, epsrel=1e-11)[0]
            for a, b in zip(edges[:-1], edges[1:]))
    return v + 2 * np.pi ** 2 / edges[-1] ** 4


def cdf_ref(x):
    """P(k lambda_max <= x) = (3 / M6) int_0^x t^2 I(t) dt (Eqs. "PDF of k", "k normalisation
    infinite"), integrated by parts: (x^3 I(x) + int_0^x t^6 phi~(t)^2 dt) / M6."""
    edges = np.concatenate([[0.0], np.arange(np.pi, x, np.pi), [x]])
    v = sum(integrate.quad(lambda t: t ** 6 * phi2(t), a, b, epsabs=0, epsrel=1e-12)[0]
            for a, b in zip(edges[:-1], edges[1:]) if b > a)
    return (x ** 3 * I_ref(x) + v) / M6


def free_pairs(O, seps, per_sep, params, spacing=50.0):
    """Tracer pairs, each pair its own infinite system (two free particles)."""
    rng = np.random.default_rng(2)
    pos, rs, dirs = [], [], []
    k = 0
    for r in seps:
        for _ in range(per_sep):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            c = np.array([k, 0.0, 0.0]) * spacing
            pos += [c - 0.5 * r * d, c + 0.5 * r * d]
            rs.append(r)
            dirs.append(d)
            k += 1
    pos = np.array(pos)
    nsys = len(rs)
    off = np.arange(nsys + 1) * 2
    return O.Oracle(params, off, np.arange(2 * nsys + 1), pos), pos, np.array(rs), np.array(dirs)


# ------------------------------------------------------------------- infinite plane waves
def test_infinite_k_table_inverts_the_cdf(oracle_mod):
    p = dict(periodic=0, plane_waves=1, lambda_min=1.0, lambda_max=4.0, bond_type="none", wca=0, A0=0.5, seed=1)
    o = oracle_mod.Oracle(p, [0, 2], [0, 1, 2], np.array([[0.0, 0, 0], [3.0, 0, 0]]))
    info = o.system_info()
    assert info["P_F"] == pytest.approx(1.0 / 64.0, rel=1e-15)
    assert info["N_k"] == pytest.approx(3 * 4.0 ** 3 / M6, rel=1e-15)
    assert oracle_mod.G(0.0) == pytest.approx(M6 / 3.0, rel=1e-10)
    # the tail of the table: x v -> 2 pi^2 / G(0) as v -> 0 (I(x) ~ 2 pi^2 x^-4)
    tab = o.inf_table()
    assert tab[-1] == pytest.approx(2 * np.pi ** 2 / (M6 / 3.0), rel=1e-9)
    t = np.arange(len(tab)) / (len(tab) - 1)
    x = tab[1:-1] / (1 - t[1:-1] ** 3)
    assert tab[0] == 0.0 and np.all(np.diff(x) > 0)
    # linear interpolation in t is exact to ~1e-5 where P(k) is smooth; in the tail I(x) carries
    # wiggles of relative size ~1/x (phi~^2 oscillates like cos^2 q), which 4097 points resolve
    # only to ~1e-3 of v
    for v, rel in ((0.999, 2e-5), (0.9, 2e-5), (0.7, 2e-5), (0.5, 2e-5), (0.3, 2e-5), (0.1, 1e-4),
                   (0.02, 1e-3), (0.003, 1e-3)):
        x = o.inf_x_of_v(v)
        assert 1.0 - cdf_ref(x) == pytest.approx(v, rel=rel, abs=1e-7), (v, x)
    assert o.inf_x_of_v(1.0) == 0.0


def test_infinite_plane_wave_k_histogram(oracle_mod):
    """Free particles, plane waves only, every wave accepted: the |k| lambda_max shells of the
    trace follow the CDF of Eq. "PDF of k"."""
    N = 64
    pos = np.random.default_rng(3).uniform(0, 6.0, (N, 3))
    p = dict(periodic=0, plane_waves=1, wavelets=0, lambda_min=1.0, lambda_max=2.0, bond_type="none", wca=0,
             A0=0.5, seed=5)
    o = oracle_mod.Oracle(p, [0, N], np.arange(N + 1), pos, trace_capacity=200_000)
    o.sweep(4000)
    tr = o.trace(200_000)
    pw = tr[tr["kind"] == 2]
    assert np.all(pw["accepted"] == 1) and np.all(pw["retry"] == 0)
    assert len(pw) == pytest.approx(4000 * N / 8.0, rel=6 / np.sqrt(4000 * N / 8.0))
    edges = [0, 1, 2, 3, 4, 6, 9, 15]
    F = [cdf_ref(e) if e > 0 else 0.0 for e in edges] + [1.0]
    shell = pw["extra"]
    ob = o.observables()
    np.testing.assert_array_equal(np.bincount(shell, minlength=16), ob["pw_shell_attempts"])
    for a, b, lo, hi in zip(edges[:-1], edges[1:], F[:-2], F[1:-1]):
        got = np.sum((shell >= a) & (shell < b))
        exp = (hi - lo) * len(pw)
        assert abs(got - exp) < 4.5 * np.sqrt(exp * (1 - hi + lo)) + 1, (a, b, got, exp)
    assert abs(np.sum(shell >= 15) - (1 - F[-2]) * len(pw)) < 4.5 * np.sqrt((1 - F[-2]) * len(pw)) + 1


def relative_moments(o, pos, dirs, S):
    """Per-sweep second moments of the relative displacement of each pair, along and across the
    pair axis (the self terms cancel, so the heavy tails of small-k plane waves drop out)."""
    par = np.zeros((S, len(dirs)))
    per = np.zeros((S, len(dirs)))
    dtau = np.zeros(S)
    for s in range(S):
        o.set_positions(pos)
        t0 = o.tau().sum()
        o.set_sweep(s)
        o.sweep(1)
        dtau[s] = o.tau().sum() - t0
        d = o.positions() - pos
        rel = d[1::2] - d[0::2]
        a = np.sum(rel * dirs, 1)
        par[s] = a * a
        per[s] = (np.sum(rel * rel, 1) - a * a) / 2
    return par, per, dtau


@pytest.mark.parametrize("plane_waves", [0, 1])
def test_infinite_plane_waves_complete_the_oseen_tail(oracle_mod, plane_waves):
    """Relative motion of two free tracers per sweep, 2 (s - c(r)) along and across the pair axis,
    with s the self term and c(r) = (3 N_lambda / 16 pi^2) A0^2 O_w(r): O_w over
    [lambda_min, lambda_max] for wavelets alone and over [lambda_min, infinity) once the plane
    waves of the infinite system are added (Eqs. "R^inf definition", "P(Fourier) infinite");
    then also tau per sweep is N dt of Eq. "dt w+F", so that s = a^2 tau per sweep: free particles
    diffuse with D0 = a^2/(6 tau) whatever lambda_max is (Sec. VI.C)."""
    lmin, lmax, A0 = 1.0, 3.0, 0.2
    seps = [0.75, 1.5, 3.0, 5.0, 8.0]
    p = dict(periodic=0, plane_waves=plane_waves, lambda_min=lmin, lambda_max=lmax, bond_type="none", wca=0,
             A0=A0, seed=13 + plane_waves)
    o, pos, rs, dirs = free_pairs(oracle_mod, seps, 48, p)
    S = 1500
    par, per, dtau = relative_moments(o, pos, dirs, S)
    # with the plane waves, (1 - P_F) N_lambda = 3 lambda_min^3 and lambda_max drops out
    nl = 3 * lmin ** 3 if plane_waves else 3 / (lmin ** -3 - lmax ** -3)
    pref = 3 * nl / (16 * np.pi ** 2) * A0 ** 2
    # self term per sweep and component (Eq. "wavelet dr2" times the N moves of a sweep)
    s3 = 2 * A0 ** 2 * M4 * nl * (1 / lmin - (0.0 if plane_waves else 1 / lmax)) / (2 * np.pi) ** 3 / 3
    for r in seps:
        m = rs == r
        a = np.array(Ow_components(r, lmin)) - (0 if plane_waves else np.array(Ow_components(r, lmax)))
        for meas, pred in ((par[:, m], 2 * (s3 - pref * a[0])), (per[:, m], 2 * (s3 - pref * a[1]))):
            err = meas.std() / np.sqrt(meas.size)
            assert abs(meas.mean() - pred) < 4.5 * err + 0.01 * pred, (plane_waves, r, meas.mean(), pred, err)
    if plane_waves:
        nsys = len(rs)
        tau_sweep = 6 * A0 ** 2 * M4 * LAM_A ** 2 / (8 * np.pi ** 3)  # N dt, Eq. "dt w+F"
        assert dtau.mean() / nsys == pytest.approx(tau_sweep, rel=0.01)
        assert 3 * s3 == pytest.approx((lmin / LAM_A) ** 2 * tau_sweep, rel=1e-12)


# --------------------------------------------------------------------------------- Glauber
def test_glauber_acceptance_function(oracle_mod):
    """Accepted fraction of the tests of a sweep, binned in dU, follows 1/(1 + exp(dU/kT))."""
    from paper_1611_09160_amd import workloads as W

    sysd = W.make_solution(n_chains=24, n_beads=16, box_L=10.0, seed=5)
    p = dict(periodic=1, plane_waves=1, box_L=10.0, lambda_min=1.0, lambda_max=2.5, bond_type="fene",
             k_bond=30.0, R0=1.5, wca=1, A0=0.9, kT=1.0, seed=61, accept="glauber")
    o = oracle_mod.Oracle(p, [0, len(sysd["pos"])], sysd["chain_offset"], sysd["pos"], trace_capacity=3_000_000)
    o.sweep(20)
    tr = o.trace(3_000_000)
    t = tr[(tr["kind"] != 1) & np.isfinite(tr["dU"]) & (tr["n"] > 0)]
    np.testing.assert_allclose(t["thr"] >= t["dU"], t["accepted"] == 1)
    edges = np.array([-3, -1.5, -0.75, -0.25, 0.25, 0.75, 1.5, 3])
    for a, b in zip(edges[:-1], edges[1:]):
        m = (t["dU"] >= a) & (t["dU"] < b)
        assert m.sum() >= 300, (a, b, m.sum())
        pred = np.mean(1 / (1 + np.exp(t["dU"][m])))
        got = t["accepted"][m].mean()
        assert abs(got - pred) < 4.5 * np.sqrt(pred * (1 - pred) / m.sum()) + 0.003, (a, b, got, pred, m.sum())


# ------------------------------------------------------------------------ uniform centring
def test_uniform_centring_gives_the_same_correlations(oracle_mod):
    """b uniform in the box with A_w = A0 lambda / sqrt(<n>) gives the two-tracer correlations
    of the anchored scheme, (3 N_lambda / 16 pi^2) O_w(r; lambda_min, lambda_max) per sweep."""
    lmin, lmax, A0, L = 1.0, 3.0, 0.2, 30.0
    seps = [0.75, 1.5, 3.0, 5.0]
    rng = np.random.default_rng(4)
    pos, rs, dirs = [], [], []
    # pairs on a lattice of spacing 7.5 (> 2 lambda_max): 4^3 = 64 pairs in the box
    g = np.arange(4) * 7.5 + 2.0
    for i, c in enumerate(np.array(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1).T):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        r = seps[i % len(seps)]
        pos += [c - 0.5 * r * d, c + 0.5 * r * d]
        rs.append(r)
        dirs.append(d)
    pos, rs, dirs = np.array(pos), np.array(rs), np.array(dirs)
    N = len(pos)
    p = dict(periodic=1, plane_waves=0, box_L=L, lambda_min=lmin, lambda_max=lmax, bond_type="none", wca=0,
             A0=A0, seed=29, centring="uniform")
    o = oracle_mod.Oracle(p, [0, N], np.arange(N + 1), pos)
    S = 1200
    par = np.zeros((S, len(rs)))
    per = np.zeros((S, len(rs)))
    self_ = np.zeros((S, len(rs)))
    for s in range(S):
        o.set_positions(pos)
        o.set_sweep(s)
        o.sweep(1)
        d = o.positions() - pos
        d1, d2 = d[0::2], d[1::2]
        p1, p2 = np.sum(d1 * dirs, 1), np.sum(d2 * dirs, 1)
        par[s] = p1 * p2
        per[s] = (np.sum(d1 * d2, 1) - p1 * p2) / 2
        self_[s] = np.sum(d1 * d1, 1)
    nl = 3 / (lmin ** -3 - lmax ** -3)
    pref = 3 * nl / (16 * np.pi ** 2) * A0 ** 2
    for r in seps:
        m = rs == r
        a, b = np.array(Ow_components(r, lmin)), np.array(Ow_components(r, lmax))
        for meas, pred in ((par[:, m], pref * (a[0] - b[0])), (per[:, m], pref * (a[1] - b[1]))):
            err = meas.std() / np.sqrt(meas.size)
            assert abs(meas.mean() - pred) < 4.5 * err + 2e-6, (r, meas.mean(), pred, err)
    pred_self = 2 * A0 ** 2 * M4 * nl * (1 / lmin - 1 / lmax) / (2 * np.pi) ** 3
    assert self_.mean() == pytest.approx(pred_self, rel=4.5 * self_.std() / np.sqrt(self_.size) / pred_self)
    ob = o.observables()
    # every trial centre lies in its cell, and moves without particles (n = 0) are accepted
    assert np.all(ob["hits"] == ob["trials"]) and np.all(ob["accepts"] == ob["attempts"])
