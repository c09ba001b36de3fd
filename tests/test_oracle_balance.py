"""Equilibrium and diffusion pins of the oracle against closed forms (CPU only).

- T9, detailed balance on three-bead chains: harmonic chains drawn exactly from the Boltzmann
  distribution, one sweep each; a move set that satisfies detailed balance leaves every
  statistic unchanged in expectation (bond lengths, bond angle, end-to-end distance, their
  histograms) and keeps E[f(X) g(X')] = E[g(X) f(X')]. Exact for the rotation map of the
  wavelet (with Metropolis or Glauber acceptance, anchored or uniform centres) and for plane
  waves, without parameter recycling (Sec. IV, Eq. "Metropolis test"). Two parts of the method
  as printed are not exactly balanced, and these checks measure it: the linear map
  x + A w(x) of Eq. "Oseen as <ww>" (its reverse move returns only to first order) stretches
  bonds, and lambda recycling (App. D "Parameter recycling") makes each proposal depend on the
  rejections before it, which favours easily accepted (compressed) states.
- T5, ideal chain: <R_g^2> = b^2 (N^2 - 1) / (6 N) for N beads (Eq. "Radius of gyration",
  Gaussian chain with <b^2> = 3 kT / k), over a run started from exact equilibrium.
- T6, chain diffusion (Sec. VI.B): with wavelets smaller than half the closest bead approach
  every move holds one bead, and the centre of mass diffuses with D0 / N, D0 = a^2/(6 tau)
  (Eq. "Unit of Time"); with larger wavelets the short-time centre-of-mass diffusion of a
  Gaussian chain is the Kirkwood sum over pairs of the wavelet mobility, (1/N^2) sum_ij
  tr D_ij / 3 with D_ij from O_w (Eqs. "Oseen (min,infty)", "Oseen_w", "D series").
"""
import numpy as np
import pytest

from tests.test_oracle_dynamics import Ow_components

M3 = 2 * np.pi ** 2 / 105 * (9 - 8 * np.log(2))
M4 = 8 * np.pi ** 3 / 105
LAM_A = 2 / np.pi * M4 / M3

HARM3 = dict(lambda_min=1.0, lambda_max=4.0, bond_type="harmonic", k_bond=3.0, wca=0, r_int_harmonic=5.0)


def boltzmann_chains(rng, nsys, nb, k):
    b = rng.normal(scale=np.sqrt(1.0 / k), size=(nsys, nb - 1, 3))
    return np.concatenate([np.zeros((nsys, 1, 3)), np.cumsum(b, 1)], 1)


def features(x, box):
    b1, b2 = x[:, 1] - x[:, 0], x[:, 2] - x[:, 1]
    if box:
        b1 = b1 - box * np.rint(b1 / box)
        b2 = b2 - box * np.rint(b2 / box)
    l1, l2 = np.sum(b1 * b1, 1), np.sum(b2 * b2, 1)
    cos = np.sum(b1 * b2, 1) / np.sqrt(l1 * l2)
    return np.stack([l1, l2, np.sum(b1 * b2, 1), np.sum((b1 + b2) ** 2, 1), np.sqrt(l1), cos], 1)


def one_sweep_statistics(oracle_mod, params, reps, seed=0, chains_per_box=0, box=0.0, nsys=4095):
    """Features of three-bead chains before and after one sweep from exact equilibrium.

    chains_per_box = 0: every chain its own infinite system; else nsys periodic boxes of side
    box holding chains_per_box independent chains each (uniform centring needs a density)."""
    rng = np.random.default_rng(seed)
    k = params["k_bond"]
    per = max(1, chains_per_box)
    nch = nsys * per

    def sample():
        r = boltzmann_chains(rng, nch, 3, k)
        if chains_per_box:
            return (r + rng.uniform(0, box, (nch, 1, 3))).reshape(-1, 3)
        return (r + 1000.0 * np.arange(nch)[:, None, None]).reshape(-1, 3)

    sys_off = np.arange(nsys + 1) * 3 * per
    chain_off = np.arange(nch + 1) * 3
    kw = dict(sys_box_L=np.full(nsys, box), sys_lambda_max=np.full(nsys, params["lambda_max"])) if box else {}
    o = oracle_mod.Oracle(params, sys_off, chain_off, sample(), **kw)
    fo, fn = [], []
    for rep in range(reps):
        pos = sample()
        o.set_positions(pos)
        o.set_sweep(rep)
        o.sweep(1)
        fo.append(features(pos.reshape(nch, 3, 3), box))
        fn.append(features(o.positions().reshape(nch, 3, 3), box))
    return np.concatenate(fo), np.concatenate(fn), o.observables()


def balance_z(fo, fn):
    """z-scores: stationarity of the features and of histogram bins, and reversibility."""
    def z(d):
        return d.mean(0) / (d.std(0) / np.sqrt(len(d)) + 1e-300)

    zs = list(z(fn[:, :4] - fo[:, :4]))
    for col, edges in ((4, np.linspace(0.2, 1.8, 9)), (5, np.linspace(-1, 1, 9))):
        io = np.digitize(fo[:, col], edges)
        ino = np.digitize(fn[:, col], edges)
        for bb in range(1, len(edges)):
            zs.append(z((ino == bb).astype(float) - (io == bb).astype(float)))
    # E[f(X) g(X')] - E[g(X) f(X')]
    for a, b in ((0, 2), (3, 0), (1, 3)):
        zs.append(z(fo[:, a] * fn[:, b] - fo[:, b] * fn[:, a]))
    return np.array(zs, dtype=float)


EXACT = {
    "rotation-metropolis": dict(periodic=0, plane_waves=0, wavelet_map="rotation", retry_cap=1, A0=1.0),
    "rotation-glauber": dict(periodic=0, plane_waves=0, wavelet_map="rotation", accept="glauber", retry_cap=1, A0=1.0),
    "infinite-plane-waves": dict(periodic=0, plane_waves=1, wavelets=0, retry_cap=1, A0=1.0, lambda_max=1.5),
    "rotation-uniform-centres": dict(periodic=1, plane_waves=0, wavelet_map="rotation", centring="uniform", retry_cap=1,
                                     A0=1.0, lambda_max=2.5),
}


@pytest.mark.parametrize("name", list(EXACT))
def test_detailed_balance_three_beads(oracle_mod, name):
    over = EXACT[name]
    p = dict(HARM3, seed=9, **over)
    if over.get("centring") == "uniform":
        fo, fn, ob = one_sweep_statistics(oracle_mod, p, 40, chains_per_box=200, box=10.0, nsys=32)
    else:
        fo, fn, ob = one_sweep_statistics(oracle_mod, p, 200)
    moved = ob["accepts"].sum() + ob["pw_accepts"]
    assert moved > 0.2 * len(fo)
    assert ob["attempts"].sum() + ob["pw_attempts"] > ob["accepts"].sum() + ob["pw_accepts"]  # rejections happen
    zs = balance_z(fo, fn)
    assert np.max(np.abs(zs)) < 4.5, (name, np.round(zs, 2))


def test_linear_wavelet_map_is_not_balanced(oracle_mod):
    """The printed linear map stretches bonds from exact equilibrium: the mean squared bond
    length grows in one sweep (the rotation map with the same draws does not, see above)."""
    p = dict(HARM3, periodic=0, plane_waves=0, wavelet_map="linear", retry_cap=1, A0=1.5, seed=9)
    fo, fn, _ = one_sweep_statistics(oracle_mod, p, 200)
    d = (fn[:, 0] + fn[:, 1]) - (fo[:, 0] + fo[:, 1])
    assert d.mean() > 6 * d.std() / np.sqrt(len(d)), (d.mean(), d.std() / np.sqrt(len(d)))


def test_lambda_recycling_is_not_balanced(oracle_mod):
    """lambda recycling with the exact rotation map compresses bonds from exact equilibrium."""
    p = dict(HARM3, periodic=0, plane_waves=0, wavelet_map="rotation", retry_cap=64, A0=1.5, seed=9)
    fo, fn, ob = one_sweep_statistics(oracle_mod, p, 200)
    d = (fn[:, 0] + fn[:, 1]) - (fo[:, 0] + fo[:, 1])
    assert d.mean() < -6 * d.std() / np.sqrt(len(d)), (d.mean(), d.std() / np.sqrt(len(d)))
    assert ob["attempts"].sum() > ob["hits"].sum()


# ------------------------------------------------------------------------------ T5: R_g^2
def rg2_run(oracle_mod, params, nch=256, nb=64, sweeps=150, seed=4):
    rng = np.random.default_rng(seed)
    r = boltzmann_chains(rng, nch, nb, params["k_bond"]) + 3000.0 * np.arange(nch)[:, None, None]
    off = np.arange(nch + 1) * nb
    o = oracle_mod.Oracle(params, off, off, r.reshape(-1, 3))
    start = o.chain_rg2()
    traj = []
    for _ in range(sweeps):
        o.sweep(1)
        traj.append(o.chain_rg2())
    return start, np.array(traj), o.observables()


@pytest.mark.parametrize("scheme,A0", [("exact", 0.5), ("paper", 0.5), ("paper", 0.25)])
def test_ideal_chain_radius_of_gyration(oracle_mod, scheme, A0):
    """The 64-bead ideal chain (harmonic k = 3, lambda 1..16, infinite system): over 150 sweeps
    from exact equilibrium the mean R_g^2 stays at b^2 (N^2 - 1)/(6 N) = 10.664. Each chain's
    time average is one block; the paired change from the start isolates the dynamics."""
    over = dict(wavelet_map="rotation", retry_cap=1) if scheme == "exact" else dict(wavelet_map="linear", retry_cap=64)
    p = dict(periodic=0, plane_waves=0, lambda_min=1.0, lambda_max=16.0, bond_type="harmonic", k_bond=3.0, wca=0,
             r_int_harmonic=4.0, A0=A0, seed=17, **over)
    nb = 64
    exact = (nb * nb - 1) / (6.0 * nb)
    start, traj, ob = rg2_run(oracle_mod, p)
    assert ob["accepts"].sum() > 0.5 * ob["attempts"].sum()
    blocks = traj.mean(0)
    err = blocks.std() / np.sqrt(len(blocks))
    assert abs(blocks.mean() - exact) < 4.5 * err, (scheme, A0, blocks.mean(), exact, err)
    change = (traj[-50:].mean(0) - start)
    cerr = change.std() / np.sqrt(len(change))
    assert abs(change.mean()) < 4.5 * cerr, (scheme, A0, change.mean(), cerr)


# --------------------------------------------------------------------------- T6: diffusion
def test_rouse_centre_of_mass_diffusion(oracle_mod):
    """FENE + WCA 8-bead chains with lambda in [0.2, 0.35]: no wavelet holds two beads (they stay
    more than 0.7 apart), so there is no hydrodynamic coupling and D_cm = D0 / N."""
    from paper_1611_09160_amd import workloads as W

    lmin, lmax, nb, A0 = 0.2, 0.35, 8, 0.1
    p = dict(periodic=0, plane_waves=0, lambda_min=lmin, lambda_max=lmax, bond_type="fene", k_bond=30.0, R0=1.5,
             wca=1, A0=A0, seed=3)
    msd, tau = [], []
    for rep in range(3):
        chains = [W.make_solution(1, nb, 1000.0, seed=1000 * rep + i, periodic=False)["pos"] for i in range(2000)]
        pos = np.concatenate([c - c[0] + 50.0 * i for i, c in enumerate(chains)])
        off = np.arange(len(chains) + 1) * nb
        o = oracle_mod.Oracle(p, off, off, pos)
        o.sweep(5)
        c0, t0 = o.chain_com(), o.tau().copy()
        o.sweep(20)
        msd.append(np.sum((o.chain_com() - c0) ** 2, 1))
        tau.append(o.tau() - t0)
        ob = o.observables()
        assert ob["bead_updates"].sum() == ob["attempts"].sum()  # one bead per move
    msd, tau = np.concatenate(msd), np.concatenate(tau)
    a = lmin / LAM_A
    ratio = (msd.sum() / (6 * tau.sum())) * nb / (a * a / 6)
    err = (msd / tau).std() / np.sqrt(len(msd)) / (msd / tau).mean()
    # Metropolis rejections shorten the accepted steps at O(A0^2): 0.5 % at A0 = 0.1
    assert abs(ratio - 1.0) < 4.5 * err + 0.01, (ratio, err)


def test_kirkwood_short_time_diffusion(oracle_mod):
    """Gaussian 8-bead chains (harmonic k = 3, lambda 1..4), one sweep from exact equilibrium:
    centre-of-mass mean square displacement per sweep = (1/N^2) [N s + sum_{i != j} c(r_ij)] with
    s the self term (Eq. "wavelet dr2" times N moves) and c(r) = (3 N_lambda/16 pi^2) A0^2 tr O_w(r)
    (the Kirkwood form of Eq. "D series" with the wavelet mobility)."""
    lmin, lmax, nb, A0, nsys = 1.0, 4.0, 8, 0.1, 4095
    p = dict(HARM3, periodic=0, plane_waves=0, A0=A0, seed=7)
    rho = np.concatenate([np.linspace(0.02, 2.0, 50), np.linspace(2.05, 12.0, 60)])
    tab = np.array([Ow_components(r, 1.0) for r in rho])  # O_w(r; lam) = tab(r / lam) / lam

    def ow_trace(r, lam):
        x = np.minimum(r / lam, rho[-1])
        return (np.interp(x, rho, tab[:, 0]) + 2 * np.interp(x, rho, tab[:, 1])) / lam

    nl = 3 / (lmin ** -3 - lmax ** -3)
    pref = 3 * nl / (16 * np.pi ** 2) * A0 ** 2
    s_self = 2 * A0 ** 2 * M4 * nl * (1 / lmin - 1 / lmax) / (2 * np.pi) ** 3
    rng = np.random.default_rng(2)
    off = np.arange(nsys + 1) * nb
    iu = np.triu_indices(nb, 1)
    meas, pred = [], []
    o = None
    for rep in range(20):
        r = boltzmann_chains(rng, nsys, nb, 3.0) + 1000.0 * np.arange(nsys)[:, None, None]
        if o is None:
            o = oracle_mod.Oracle(p, off, off, r.reshape(-1, 3))
        o.set_positions(r.reshape(-1, 3))
        o.set_sweep(rep)
        o.sweep(1)
        meas.append(np.sum((o.chain_com() - r.mean(1)) ** 2, 1))
        rr = np.linalg.norm(r[:, iu[0]] - r[:, iu[1]], axis=-1)
        cross = 2 * pref * (ow_trace(rr, lmin) - ow_trace(rr, lmax)).sum(1)
        pred.append((nb * s_self + cross) / nb ** 2)
    meas, pred = np.concatenate(meas), np.concatenate(pred)
    ratio = meas.mean() / pred.mean()
    err = meas.std() / np.sqrt(len(meas)) / pred.mean()
    assert abs(ratio - 1.0) < 4.5 * err + 0.005, (ratio, err)
    # the hydrodynamic coupling is a large part of it: without the pair terms the prediction
    # would be 1/N of the self term alone
    assert pred.mean() > 2.0 * s_self / nb
