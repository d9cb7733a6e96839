"""Velocity sets and w-orthogonal moment bases (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The basis rows are built here from their defining polynomials in the discrete
velocity c_i, and the norms N_a from Sec. III eq. T-orthog
(N_a = sum_i w_i T_ai^2).  Nothing is copied from the HIP tables: the HIP side
writes its matrices out as integer literals, this side evaluates polynomials.

D2Q9 (App. B, table tab:modes-d2q9 and eq. TD2Q9):
  velocity order 0, +x, +y, -x, -y, (+,+), (-,+), (-,-), (+,-) -- the column
  order of the printed matrix; weights 4/9, 1/9, 1/36.
  rows: 1, c_x, c_y, 3c^2-2, 2c_x^2-c^2, c_x c_y, (3c^2-4)c_x, (3c^2-4)c_y,
        9c^4-15c^2+2.
  Pinned against the printed 9x9 matrix and the printed N_a column.

D3Q19 (not printed in the paper, which only cites bases in the literature):
  velocity order 0 | +x -x +y -y +z -z | xy(++ +- -+ --) | xz(...) | yz(...);
  weights 1/3, 1/18, 1/36.
  rows: 1 | c_x c_y c_z | c^2-1 | 3c_x^2-c^2, c_y^2-c_z^2, c_xc_y, c_yc_z, c_zc_x |
        (3c^2-5)c_a (a=x,y,z) | (c_y^2-c_z^2)c_x, (c_z^2-c_x^2)c_y, (c_x^2-c_y^2)c_z |
        3c^4-6c^2+1 | (2c^2-3)(3c_x^2-c^2) | (2c^2-3)(c_y^2-c_z^2).
  Pinned by w-orthogonality, completeness (Sec. III eqs. T-orthog, T-complete),
  lattice isotropy and the equilibrium having no ghost projection.
"""

import numpy as np

CS2 = 1.0 / 3.0  # sigma_s^2 of both lattices (Sec. III, after eq. feq)

# mode classes: conserved density, conserved momentum, bulk stress, shear
# stress, ghost (App. B: the first d+1 rows are conserved, then transport, then
# ghost modes).
RHO, MOM, BULK, SHEAR, GHOST = "rho", "j", "bulk", "shear", "ghost"


class Lattice:
    """A DdQq velocity set with its moment basis.

    Attributes: name, d, q, c (q x 3 int, z column zero in 2-D), w (q),
    T (q x q float, rows are basis vectors), N (q), classes (list of q str).
    """

    def __init__(self, name, d, c, w, rows, classes):
        self.name = name
        self.d = d
        self.c = np.asarray(c, dtype=np.int64)
        self.q = self.c.shape[0]
        self.w = np.asarray(w, dtype=np.float64)
        self.T = np.asarray(rows, dtype=np.float64)
        self.N = (self.T ** 2 * self.w[None, :]).sum(axis=1)  # eq. T-orthog
        self.classes = list(classes)
        assert self.T.shape == (self.q, self.q)
        assert len(self.classes) == self.q

    @property
    def Tinv(self):
        """(T^-1)_{ia} = w_i T_ai / N_a  (Sec. III, after eq. T-complete)."""
        return self.w[:, None] * self.T.T / self.N[None, :]

    def noncons(self):
        """Indices of the non-conserved modes, in basis order."""
        return [a for a, k in enumerate(self.classes) if k not in (RHO, MOM)]


def d2q9():
    c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
         (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    ca = np.asarray(c, dtype=np.float64)
    cx, cy = ca[:, 0], ca[:, 1]
    c2 = cx ** 2 + cy ** 2
    rows = [
        np.ones(9), cx, cy,
        3 * c2 - 2,
        2 * cx ** 2 - c2,
        cx * cy,
        (3 * c2 - 4) * cx,
        (3 * c2 - 4) * cy,
        9 * c2 ** 2 - 15 * c2 + 2,
    ]
    classes = [RHO, MOM, MOM, BULK, SHEAR, SHEAR, GHOST, GHOST, GHOST]
    return Lattice("D2Q9", 2, c, w, rows, classes)


def d3q19():
    c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for (a, b) in ((0, 1), (0, 2), (1, 2)):
        for (sa, sb) in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
            v = [0, 0, 0]
            v[a], v[b] = sa, sb
            c.append(tuple(v))
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    ca = np.asarray(c, dtype=np.float64)
    cx, cy, cz = ca[:, 0], ca[:, 1], ca[:, 2]
    c2 = cx ** 2 + cy ** 2 + cz ** 2
    rows = [
        np.ones(19), cx, cy, cz,
        c2 - 1,
        3 * cx ** 2 - c2, cy ** 2 - cz ** 2, cx * cy, cy * cz, cz * cx,
        (3 * c2 - 5) * cx, (3 * c2 - 5) * cy, (3 * c2 - 5) * cz,
        (cy ** 2 - cz ** 2) * cx, (cz ** 2 - cx ** 2) * cy, (cx ** 2 - cy ** 2) * cz,
        3 * c2 ** 2 - 6 * c2 + 1,
        (2 * c2 - 3) * (3 * cx ** 2 - c2),
        (2 * c2 - 3) * (cy ** 2 - cz ** 2),
    ]
    classes = [RHO, MOM, MOM, MOM, BULK] + [SHEAR] * 5 + [GHOST] * 9
    return Lattice("D3Q19", 3, c, w, rows, classes)


def get(name):
    return {"D2Q9": d2q9, "D3Q19": d3q19}[name]()
