"""Seeded nuclei: charges Z_k and positions R_k (atomic units).

Draw order for one system from numpy's PCG64 generator ``rng``:
  1. charges: Z ~ U{1..z_max} for every nucleus, redrawn as a whole until
     sum(Z) >= min_charge;
  2. positions, nucleus by nucleus: R ~ U[-r, r]^3, redrawn until it is at
     least min_spacing away from every nucleus already placed.
"""
from dataclasses import dataclass
import numpy as np


@dataclass
class Atoms:
    Z: np.ndarray   # [M] float64
    R: np.ndarray   # [M][3] float64

    @property
    def M(self):
        return self.Z.shape[0]


def sample_atoms(rng, n_atoms, z_max, min_charge, box, min_spacing=None):
    while True:
        Z = rng.integers(1, z_max + 1, size=n_atoms).astype(np.float64)
        if Z.sum() >= min_charge:
            break
    R = []
    for _ in range(n_atoms):
        for _tries in range(100000):
            r = rng.uniform(-box, box, size=3)
            if min_spacing is None or all(np.linalg.norm(r - q) >= min_spacing for q in R):
                R.append(r)
                break
        else:
            raise RuntimeError("could not place nuclei with the requested spacing")
    return Atoms(Z=Z, R=np.array(R, dtype=np.float64).reshape(-1, 3))
