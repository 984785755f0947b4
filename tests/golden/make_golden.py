"""Writes the closed-form reference values stored next to this script (no GPU, no oracle state).

Run: python tests/golden/make_golden.py   (prints the table; compare with the stored file)
"""
import math

C = 137.036


def dirac_coulomb(n, kappa, Z=1.0, c=C):
    g = math.sqrt(kappa * kappa - (Z / c) ** 2)
    return c * c / math.sqrt(1.0 + (Z / c) ** 2 / (n - abs(kappa) + g) ** 2) - c * c


if __name__ == "__main__":
    for n, k, lab in [(1, -1, "1s1/2"), (2, -1, "2s1/2"), (2, 1, "2p1/2"), (2, -2, "2p3/2"),
                      (3, -1, "3s1/2"), (3, 2, "3d3/2"), (3, -3, "3d5/2")]:
        print(n, k, lab, repr(dirac_coulomb(n, k)))
