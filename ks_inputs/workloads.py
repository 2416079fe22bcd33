"""The five synthetic workloads (and reduced-size variants for parity tests).

Each stands in for a molecule of the paper's experiments (Sec. 4: He, LiH,
CH4, C6H6 on adaptive P1 meshes of 9e3 .. 2.8e6 elements in a cube of side
20 Bohr, 1 .. 21 doubly occupied orbitals).  The paper's adaptive meshes are
not available, so a structured Kuhn mesh moved toward the sampled nuclei
replaces them.

  hydrogen         P1, 16^3 hexes, [-10,10]^3, Z=1 at the origin, k=1, f=[1],
                   no Hartree / XC, unmoved mesh, coarse n_H=4
  small_molecule   P2, 32^3, [-15,15]^3, seed 2: 3 nuclei, Z~U{1..8} with
                   sum Z >= 10, R~U[-2,2]^3, moved mesh, k=5, f=2, LDA, n_H=6
  mixed            P2, 64^3, [-15,15]^3, seed 3: 10 nuclei, Z~U{1..8} with
                   sum Z >= 48, R~U[-5,5]^3 spacing >= 1.5, moved, k=24, n_H=6
  batched          48 systems, seeds 4000+s: n~U{12..40}, order~U{1,2},
                   1..6 nuclei Z~U{1..8}, R~U[-3,3]^3 spacing >= 1.5, [-12,12]^3,
                   k~U{1..min(12, sum Z // 2)}, moved, n_H = 4 if n < 24 else 6
  differentiation  P1, 96^3, [-12,12]^3, seed 5: 20 nuclei Z~U{1..6} with
                   sum Z >= 80, R~U[-6,6]^3 spacing >= 1.5, unmoved, k=40, n_H=6
  lih, ch4, c6h6   the paper's molecules (positions and charges from Sec. 4),
                   [-10,10]^3, P1 by default, n^3 hexes moved toward the
                   nuclei, k = 2, 5, 21, LDA, n_H = 4 if n < 24 else 6
"""
from dataclasses import dataclass, field
import numpy as np

from .mesh import Mesh, freudenthal_mesh, move_nodes_toward_nuclei
from .quadrature import QuadRule, rule_for_order
from .atoms import Atoms, sample_atoms


@dataclass
class Workload:
    name: str
    mesh: Mesh
    quad: QuadRule
    atoms: Atoms
    k: int                     # number of orbitals (right-hand sides)
    occ: np.ndarray            # [k] occupations
    n_H: int                   # coarse hexes per side
    hartree: bool              # Hartree potential on/off
    xc: bool                   # LDA exchange-correlation on/off
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def mu_paper(self):
        """Shift of the experiments (Sec. 4): 8 M sum_k Z_k^2."""
        return 8.0 * self.atoms.M * float(np.sum(self.atoms.Z ** 2))


WORKLOADS = ("hydrogen", "small_molecule", "mixed", "batched", "differentiation", "lih", "ch4", "c6h6")

_FULL_N = {"hydrogen": 16, "small_molecule": 32, "mixed": 64, "differentiation": 96}


def _build(name, order, n, L, atoms, k, occ, n_H, hartree, xc, moved, seed, extra=None):
    mesh = freudenthal_mesh(n, L, order)
    if moved:
        mesh = move_nodes_toward_nuclei(mesh, atoms.R)
    return Workload(name=name, mesh=mesh, quad=rule_for_order(order), atoms=atoms, k=k,
                    occ=np.asarray(occ, dtype=np.float64), n_H=n_H, hartree=hartree,
                    xc=xc, seed=seed, extra=extra or {})


def make_workload(name: str, n: int = None, k: int = None, system: int = 0,
                  order: int = None) -> Workload:
    """Build a workload; ``n``/``k``/``order`` override the mesh size, the
    orbital count and the element order for reduced parity cases (the nuclei
    are drawn exactly as for the full-size workload)."""
    if name == "hydrogen":
        atoms = Atoms(Z=np.array([1.0]), R=np.zeros((1, 3)))
        kk = k or 1
        occ = [1.0] * kk
        return _build(name, order or 1, n or 16, 10.0, atoms, kk, occ, 4, False, False,
                      False, 0)
    if name == "small_molecule":
        rng = np.random.default_rng(2)
        atoms = sample_atoms(rng, 3, 8, 10, 2.0)
        kk = k or 5
        return _build(name, order or 2, n or 32, 15.0, atoms, kk, [2.0] * kk, 6, True, True,
                      True, 2)
    if name == "mixed":
        rng = np.random.default_rng(3)
        atoms = sample_atoms(rng, 10, 8, 48, 5.0, 1.5)
        kk = k or 24
        return _build(name, order or 2, n or 64, 15.0, atoms, kk, [2.0] * kk, 6, True, True,
                      True, 3)
    if name == "differentiation":
        rng = np.random.default_rng(5)
        atoms = sample_atoms(rng, 20, 6, 80, 6.0, 1.5)
        kk = k or 40
        return _build(name, order or 1, n or 96, 12.0, atoms, kk, [2.0] * kk, 6, True, True,
                      False, 5)
    if name in ("lih", "ch4", "c6h6"):
        from .molecules import molecule, BOX_HALF
        atoms, kk = molecule(name)
        kk = k or kk
        return _build(name, order or 1, n or 32, BOX_HALF, atoms, kk, [2.0] * kk,
                      4 if (n or 32) < 24 else 6, True, True, True, 0)
    if name == "batched":
        s = int(system)
        rng = np.random.default_rng(4000 + s)
        nn = int(rng.integers(12, 41))
        oo = int(rng.integers(1, 3))
        M = int(rng.integers(1, 7))
        atoms = sample_atoms(rng, M, 8, 2, 3.0, 1.5)
        kmax = int(min(12, atoms.Z.sum() // 2))
        kk = int(rng.integers(1, kmax + 1))
        if k is not None:
            kk = k
        n_use = n or nn
        return _build(f"batched[{s}]", order or oo, n_use, 12.0, atoms, kk, [2.0] * kk,
                      4 if n_use < 24 else 6, True, True, True, 4000 + s)
    raise KeyError(name)


def batched_systems(count: int = 48, n_cap: int = None):
    """All systems of the batched workload; ``n_cap`` limits the mesh size for
    quick parity runs."""
    out = []
    for s in range(count):
        w = make_workload("batched", system=s)
        if n_cap is not None and w.mesh.n > n_cap:
            w = make_workload("batched", system=s, n=n_cap)
        out.append(w)
    return out
