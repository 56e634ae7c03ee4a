"""Seeded synthetic workloads (inputs only: no discretisation or solver arithmetic here).

Both the GPU library and the CPU oracle receive exactly these numbers (mode lists, sizes,
options), so their results can be compared.  Recipes:

  heat-p2-h16-Nt128      unit square, kappa 1, T 0.1, N_t 128, p 2, h 2^-4, two-level MGRIT m 4;
                         manufactured u = sin(pi x) sin(pi y) e^{-t}: source mode (1,1) with
                         amplitude 2 pi^2 kappa - 1 and time factor e^{-t}, u0 = L2 projection of
                         sin(pi x) sin(pi y).
  heat-p{3,4,5}-h64-Nt1024  unit square, kappa 1, T 0.1, N_t 1024, h 2^-6, m 8, levels down to <= 8
                         intervals; source = 8 distinct modes sin(k pi x) sin(l pi y), (k,l) drawn
                         uniformly from {1..6}^2 without repetition, amplitudes N(0,1), seed 2107;
                         u0 = 0, constant in time.
  heat-p4-h128-Nt2048    as above with p 4, h 2^-7, N_t 2048.
  heat-p3-h64-Nt4096     as above with p 3, h 2^-6, N_t 4096.
  hetero-16              16 instances, seed 5: h from {2^-5..2^-8}, p from {2..5}, kappa log-uniform
                         in [0.1, 10], 8 on the unit square and 8 on the quarter annulus (modes in
                         parameter coordinates), N_t 1024, m 8.
"""
from __future__ import annotations

import numpy as np


def random_modes(seed: int, n_modes: int = 8, kmax: int = 6):
    rng = np.random.default_rng(seed)
    pairs = [(k, l) for k in range(1, kmax + 1) for l in range(1, kmax + 1)]
    sel = rng.choice(len(pairs), n_modes, replace=False)
    amps = rng.standard_normal(n_modes)
    return [(int(pairs[i][0]), int(pairs[i][1]), float(a)) for i, a in zip(sel, amps)]


def net_init(seed: int, zero_last: bool = False):
    """Seeded initial parameters of the warm-start network (flat float64 array, layer by layer:
    weights [cout][cin][3][3] then bias [cout], channels 3 -> 32 -> 32 -> 32 -> 1): He-scaled normal
    weights (the last layer scaled by 0.1, or zero with zero_last), zero biases."""
    rng = np.random.default_rng(seed)
    ch = [3, 32, 32, 32, 1]
    parts = []
    for l in range(4):
        ci, co = ch[l], ch[l + 1]
        w = rng.standard_normal(co * ci * 9) * np.sqrt(2.0 / (9 * ci))
        if l == 3:
            w = np.zeros_like(w) if zero_last else 0.1 * w
        parts += [w, np.zeros(co)]
    return np.concatenate(parts)


def manufactured(kappa: float = 1.0):
    """source modes, time kind and initial modes of u = sin(pi x) sin(pi y) e^{-t}"""
    return [(1, 1, 2.0 * np.pi ** 2 * kappa - 1.0)], 1, [(1, 1, 1.0)]


def config(name: str):
    """dict(instances=[dict(p, n, domain, kappa, T, Nt, src, tkind, init)], m, max_levels, coarsest_max)"""
    if name == "heat-p2-h16-Nt128":
        src, tk, init = manufactured(1.0)
        inst = [dict(p=2, n=16, domain=0, kappa=1.0, T=0.1, Nt=128, src=src, tkind=tk, init=init)]
        return dict(instances=inst, m=4, max_levels=2, coarsest_max=1)
    if name.startswith("heat-p") and name.count("-") == 3:
        _, ps, hs, nts = name.split("-")
        p, n, Nt = int(ps[1:]), int(hs[1:]), int(nts[2:])
        inst = [dict(p=p, n=n, domain=0, kappa=1.0, T=0.1, Nt=Nt, src=random_modes(2107), tkind=0, init=[])]
        return dict(instances=inst, m=8, max_levels=12, coarsest_max=8)
    if name == "hetero-16":
        rng = np.random.default_rng(5)
        inst = []
        for i in range(16):
            n = int(2 ** rng.integers(5, 9))
            p = int(rng.integers(2, 6))
            kappa = float(np.exp(rng.uniform(np.log(0.1), np.log(10.0))))
            inst.append(dict(p=p, n=n, domain=0 if i < 8 else 1, kappa=kappa, T=0.1, Nt=1024,
                             src=random_modes(5000 + i), tkind=0, init=[]))
        return dict(instances=inst, m=8, max_levels=12, coarsest_max=8)
    raise KeyError(name)


def small(name: str, p: int, n: int, Nt: int, domain: int = 0, kappa: float = 1.0, seed: int = 7):
    """a small random-mode instance for parity tests"""
    inst = [dict(p=p, n=n, domain=domain, kappa=kappa, T=0.1, Nt=Nt, src=random_modes(seed, 4, 4), tkind=0,
                 init=random_modes(seed + 1, 2, 3))]
    return dict(instances=inst, m=4, max_levels=12, coarsest_max=4)
