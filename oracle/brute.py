"""Exact-rational brute force of the 25-point star (paper's Eq. 3).

TEST INFRASTRUCTURE ONLY.  Pure Python, no arrays with halos: each neighbour
is looked up with an explicit bounds check, and points outside the interior
read the supplied boundary function (zero for the Dirichlet problem).  Used on
tiny grids to pin the C oracle.
"""

from __future__ import annotations

from fractions import Fraction


def star25(u, coeffs, boundary=lambda x, y, z: 0):
    """u: nested lists u[z][y][x] of Fractions/ints; coeffs: dict with centre
    and per-axis lists of 4 (Fractions or ints).  Returns nested lists."""
    nz, ny, nx = len(u), len(u[0]), len(u[0][0])

    def val(x, y, z):
        if 0 <= x < nx and 0 <= y < ny and 0 <= z < nz:
            return u[z][y][x]
        return boundary(x, y, z)

    out = []
    for z in range(nz):
        plane = []
        for y in range(ny):
            row = []
            for x in range(nx):
                s = Fraction(coeffs["center"]) * val(x, y, z)
                for m in range(1, 5):
                    s += Fraction(coeffs["ax"][m - 1]) * (val(x + m, y, z) + val(x - m, y, z))
                    s += Fraction(coeffs["ay"][m - 1]) * (val(x, y + m, z) + val(x, y - m, z))
                    s += Fraction(coeffs["az"][m - 1]) * (val(x, y, z + m) + val(x, y, z - m))
                row.append(s)
            plane.append(row)
        out.append(plane)
    return out
