"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds starting conformations and run parameters; it holds none of the
method's arithmetic and is used both by the HIP path's callers and by the tests that feed
the same arrays to the oracle.

Recipes:
- bead-spring chains by self-avoiding random walk: bond length 0.97 sigma, a step is
  redrawn while any earlier bead lies within 0.85 sigma (minimum image in a periodic box);
  first beads uniform in the box;
- Gaussian chains (harmonic bonds, zero rest length): steps with variance kT/k per axis;
- box sizes at a target c/c* with c* = 3 N_b / (4 pi R_g^3) and R_g of the good-solvent chain
  estimated as 0.44 N_b^0.588 sigma (a Kremer-Grest-like estimate).
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 1611091600

KG = dict(bond_type="fene", k_bond=30.0, R0=1.5, wca=1, sigma=1.0, eps=1.0, kT=1.0, A0=0.5,
          lambda_min=1.0, band_ratio=2.0, n_layers=15, retry_cap=64)


def _cell_key(p, h, n):
    return tuple((np.floor(p / h).astype(np.int64) % n).tolist())


def make_solution(n_chains: int, n_beads, box_L: float, seed: int, bond: float = 0.97,
                  min_dist: float = 0.85, periodic: bool = True) -> dict:
    """Self-avoiding random-walk chains in a periodic box. ``n_beads`` is an int or a list."""
    rng = np.random.default_rng(seed)
    lens = [int(n_beads)] * n_chains if np.isscalar(n_beads) else [int(v) for v in n_beads]
    N = int(sum(lens))
    pos = np.empty((N, 3))
    L = float(box_L)
    ncell = max(1, int(L // min_dist))
    h = L / ncell
    grid: dict = {}
    md2 = min_dist * min_dist

    def free(p):
        c = np.floor(p / h).astype(np.int64)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    key = ((c[0] + dx) % ncell, (c[1] + dy) % ncell, (c[2] + dz) % ncell)
                    for j in grid.get(key, ()):
                        d = pos[j] - p
                        if periodic:
                            d -= L * np.rint(d / L)
                        if d @ d < md2:
                            return False
        return True

    i = 0
    offsets = [0]
    for n in lens:
        # a walk that traps its own end is withdrawn and regrown from a new start
        for restart in range(100):
            start = i
            ok = True
            for b in range(n):
                for attempt in range(10000):
                    if b == 0:
                        p = rng.uniform(0.0, L, 3)
                    else:
                        u = rng.normal(size=3)
                        p = pos[i - 1] + bond * u / np.linalg.norm(u)
                    if free(p):
                        break
                else:
                    ok = False
                    break
                pos[i] = p
                grid.setdefault(_cell_key(p, h, ncell), []).append(i)
                i += 1
            if ok:
                break
            for j in range(start, i):
                grid[_cell_key(pos[j], h, ncell)].remove(j)
            i = start
        else:
            raise RuntimeError("random walk stuck: box too dense")
        offsets.append(i)
    return {"pos": pos, "chain_offset": np.array(offsets, dtype=np.int64), "box_L": L}


def gaussian_chain(n_beads: int, k_bond: float, kT: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    steps = rng.normal(scale=math.sqrt(kT / k_bond), size=(n_beads - 1, 3))
    return np.vstack([np.zeros(3), np.cumsum(steps, 0)])


def box_for(n_chains: int, n_beads: int, c_over_cstar: float) -> float:
    rg = 0.44 * n_beads ** 0.588
    cstar = 3.0 * n_beads / (4.0 * math.pi * rg ** 3)
    return (n_chains * n_beads / (c_over_cstar * cstar)) ** (1.0 / 3.0)


def config(index: int, scale: float = 1.0, seed: int | None = None) -> dict:
    """The benchmark workloads (1-based index) with run parameters and a starting state.

    ``scale`` < 1 shrinks a workload for quick parity tests (fewer chains / beads).
    """
    seed = BASE_SEED + index if seed is None else seed
    if index == 1:
        nb = max(4, int(round(64 * scale)))
        pos = gaussian_chain(nb, 3.0, 1.0, seed)
        params = dict(KG, periodic=0, plane_waves=0, bond_type="harmonic", k_bond=3.0, wca=0,
                      lambda_max=16.0, r_int_harmonic=4.0, seed=seed)
        return dict(name=f"ideal chain {nb} beads, harmonic k=3, infinite, lambda 1..16, no plane waves",
                    params=params, pos=pos, chain_offset=np.array([0, nb]), sys_offset=np.array([0, nb]))
    if index == 2:
        nb = max(16, int(round(1024 * scale)))
        L = 128.0 if scale >= 1 else max(24.0, 128.0 * scale ** (1 / 3))
        s = make_solution(1, nb, L, seed)
        params = dict(KG, periodic=1, plane_waves=1, box_L=L, lambda_max=L / 4, seed=seed)
        return dict(name=f"dilute chain {nb} beads, FENE+WCA, periodic L={L:g}, lambda 1..L/4, plane waves",
                    params=params, pos=s["pos"], chain_offset=s["chain_offset"], sys_offset=np.array([0, nb]))
    if index == 3:
        nch = max(4, int(round(256 * scale)))
        nb = 128 if scale >= 0.25 else 32
        L = 84.0 if (nch == 256 and nb == 128) else round(box_for(nch, nb, 1.0), 3)
        s = make_solution(nch, nb, L, seed)
        params = dict(KG, periodic=1, plane_waves=1, box_L=L, lambda_max=L / 4, seed=seed)
        return dict(name=f"semi-dilute {nch}x{nb} beads, FENE+WCA, periodic L={L:g}, c/c*~1, lambda 1..L/4, plane waves",
                    params=params, pos=s["pos"], chain_offset=s["chain_offset"],
                    sys_offset=np.array([0, nch * nb]))
    if index == 4:
        rng = np.random.default_rng(seed)
        nsys = max(2, int(round(512 * scale)))
        pos, coff, soff, Ls = [], [0], [0], []
        for si in range(nsys):
            nb = int(np.clip(round(math.exp(rng.normal(math.log(256), 0.8))), 32, 2048))
            if scale < 1:
                nb = max(8, int(nb * scale))
            nch = int(rng.integers(1, 9))
            L = max(16.0, round(box_for(nch, nb, 1.0), 3))
            s = make_solution(nch, nb, L, seed * 7919 + si)
            pos.append(s["pos"])
            coff += list(s["chain_offset"][1:] + soff[-1])
            soff.append(soff[-1] + nch * nb)
            Ls.append(L)
        params = dict(KG, periodic=1, plane_waves=1, box_L=Ls[0], lambda_max=Ls[0] / 4, seed=seed)
        return dict(name=f"batched {nsys} systems, lognormal chain lengths, FENE+WCA, periodic, plane waves",
                    params=params, pos=np.concatenate(pos), chain_offset=np.array(coff, dtype=np.int64),
                    sys_offset=np.array(soff, dtype=np.int64), sys_box_L=np.array(Ls),
                    sys_lambda_max=np.array(Ls) / 4)
    if index == 5:
        nch = max(8, int(round(8192 * scale)))
        nb = 128
        L = 212.0 * (nch * nb / 2 ** 20) ** (1 / 3)
        s = make_solution(nch, nb, L, seed)
        params = dict(KG, periodic=1, plane_waves=1, box_L=L, lambda_max=L / 4, seed=seed)
        return dict(name=f"homogeneous {nch}x{nb} beads, FENE+WCA, periodic L={L:.3f}, c/c*~2",
                    params=params, pos=s["pos"], chain_offset=s["chain_offset"],
                    sys_offset=np.array([0, nch * nb]))
    raise ValueError(index)


def replicas(index: int, count: int, scale: float = 1.0) -> dict:
    """``count`` independent copies of workload ``index`` (each from its own starting state) as
    one batch of systems; copy 0 is ``config(index, scale)`` itself."""
    cs = [config(index, scale, seed=BASE_SEED + index + 1000 * r) for r in range(count)]
    so, co = [0], [0]
    for c in cs:
        co += list(np.asarray(c["chain_offset"][1:]) + so[-1])
        so.append(so[-1] + int(c["sys_offset"][-1]))
    return dict(name=f"{count} copies of: {cs[0]['name']}", params=cs[0]["params"],
                pos=np.concatenate([c["pos"] for c in cs]), chain_offset=np.array(co, dtype=np.int64),
                sys_offset=np.array(so, dtype=np.int64))


def batch_semidilute(n_systems: int, n_chains: int, n_beads: int = 128, seed: int | None = None) -> dict:
    """``n_systems`` independent semi-dilute solutions of ``n_chains`` x ``n_beads`` FENE + WCA
    chains, each in its own periodic box at the bead density of the 32,768-bead solution in
    L = 84 (that solution cut into smaller systems of the same chains and concentration),
    lambda 1 .. L/4, plane waves."""
    base = BASE_SEED + 30 if seed is None else seed
    pos, so, co, Ls = [], [0], [0], []
    for i in range(n_systems):
        L = round(84.0 * (n_chains * n_beads / 32768.0) ** (1.0 / 3.0), 3)
        s = make_solution(n_chains, n_beads, L, base + 7919 * i)
        pos.append(s["pos"])
        co += list(s["chain_offset"][1:] + so[-1])
        so.append(so[-1] + n_chains * n_beads)
        Ls.append(L)
    params = dict(KG, periodic=1, plane_waves=1, box_L=Ls[0], lambda_max=Ls[0] / 4, seed=base)
    return dict(name=f"{n_systems} semi-dilute systems of {n_chains}x{n_beads} beads, FENE+WCA, L={Ls[0]:g}, "
                     f"c/c*~1, lambda 1..L/4, plane waves",
                params=params, pos=np.concatenate(pos), chain_offset=np.array(co, dtype=np.int64),
                sys_offset=np.array(so, dtype=np.int64))
