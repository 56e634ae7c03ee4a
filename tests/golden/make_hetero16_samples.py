"""Writes hetero16_oracle_samples.npz: sampled steps of the oracle's sequential implicit Euler (direct
banded-Cholesky solves, the plain definition of what converged MGRIT reproduces: Sec. 3, eq:mgrit)
for every instance of the heterogeneous 16-instance batch with n >= 128 elements per direction
(h = 2^-7 and 2^-8; full trajectories of these are too large to store and too slow to recompute
inside a test).

Calls only the oracle and the seeded input recipe.  For each such instance and each sampled step k:
  norm[k]       ||U_k||_2
  vals[k, :]    U_k at NSAMP dof indices drawn with default_rng(1000 + instance)
  proj[k, :]    <w_q, U_k> for NPROJ vectors w_q = default_rng(2000 + instance).standard_normal
                (drawn in that order, one vector per q, each of length n_dof)
Run: python tests/golden/make_hetero16_samples.py   (about 20 minutes on 8 cores)
"""
from __future__ import annotations

import os
import sys
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

STEPS = [1, 2, 3, 8, 64, 256, 512, 1000, 1023, 1024]
NSAMP = 512
NPROJ = 4
OUT = os.path.join(HERE, "hetero16_oracle_samples.npz")


def sample_indices(inst: int, ndof: int) -> np.ndarray:
    return np.sort(np.random.default_rng(1000 + inst).choice(ndof, NSAMP, replace=False))


def projection_vectors(inst: int, ndof: int) -> np.ndarray:
    rng = np.random.default_rng(2000 + inst)
    return np.stack([rng.standard_normal(ndof) for _ in range(NPROJ)])


def one(inst: int):
    import oracle as O
    from paper_2107_05337_amd import workloads as W

    d = W.config("hetero-16")["instances"][inst]
    P = O.Problem(d["p"], d["n"], d["domain"])
    U = P.sequential(d["kappa"], d["T"], d["Nt"], P.load_vector(d["src"]), d["tkind"], np.zeros(P.ndof))
    idx = sample_indices(inst, P.ndof)
    Wq = projection_vectors(inst, P.ndof)
    rows = U[STEPS]
    return inst, np.linalg.norm(rows, axis=1), rows[:, idx], rows @ Wq.T


def main():
    from paper_2107_05337_amd import workloads as W

    insts = [i for i, d in enumerate(W.config("hetero-16")["instances"]) if d["n"] >= 128]
    with Pool(min(len(insts), os.cpu_count() or 1)) as pool:
        res = sorted(pool.map(one, insts))
    out = {"instances": np.array(insts, dtype=np.int32), "steps": np.array(STEPS, dtype=np.int32)}
    for inst, nrm, vals, proj in res:
        out[f"norm_{inst}"] = nrm
        out[f"vals_{inst}"] = vals
        out[f"proj_{inst}"] = proj
    np.savez_compressed(OUT, **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
