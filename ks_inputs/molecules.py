"""The molecules of the paper's experiments (Sec. 4), as fixed inputs.

Positions in Bohr and nuclear charges, copied from the paper: lithium
hydride (the text of the LiH example: Li at (-1.0075, 0, 0), H at
(2.0075, 0, 0)), methane (the table of atomic positions in the methane
example) and benzene (the table in the benzene example).  All three are
computed in the box (-10, 10)^3 with doubly occupied orbitals: 2, 5 and
21 of them.  Data only: no part of the method.
"""
import numpy as np

from .atoms import Atoms

_LIH = [(3.0, (-1.0075, 0.0, 0.0)), (1.0, (2.0075, 0.0, 0.0))]

_CH4 = [(6.0, (0.0000, 0.0000, 0.0000)),
        (1.0, (1.3092, 1.3092, 1.3092)),
        (1.0, (-1.3092, -1.3092, 1.3092)),
        (1.0, (1.3092, -1.3092, -1.3092)),
        (1.0, (-1.3092, 1.3092, -1.3092))]

_C6H6 = [(6.0, (0.0000, 1.3970, 0.0000)),
         (6.0, (1.2098, 0.6985, 0.0000)),
         (6.0, (1.2098, -0.6985, 0.0000)),
         (6.0, (0.0000, -1.3970, 0.0000)),
         (6.0, (-1.2098, -0.6985, 0.0000)),
         (6.0, (-1.2098, 0.6985, 0.0000)),
         (1.0, (0.0000, 2.4810, 0.0000)),
         (1.0, (2.1486, 1.2405, 0.0000)),
         (1.0, (2.1486, -1.2405, 0.0000)),
         (1.0, (0.0000, -2.4810, 0.0000)),
         (1.0, (-2.1486, -1.2405, 0.0000)),
         (1.0, (-2.1486, 1.2405, 0.0000))]

MOLECULES = {"lih": (_LIH, 2), "ch4": (_CH4, 5), "c6h6": (_C6H6, 21)}
BOX_HALF = 10.0


def molecule(name):
    """(Atoms, number of doubly occupied orbitals) of a paper molecule."""
    table, k = MOLECULES[name]
    Z = np.array([z for z, _ in table], dtype=np.float64)
    R = np.array([r for _, r in table], dtype=np.float64)
    return Atoms(Z=Z, R=R), k
