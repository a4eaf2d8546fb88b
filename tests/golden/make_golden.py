"""Writes the golden closed-form fixtures in this folder.

free_electron_c1.txt: with V = 0 and D = 0 the plane-wave Hamiltonian of the
KS equation in the plane-wave basis (Sec. III.A) is diagonal, (H psi)(G) =
|k+G|^2 psi(G) in Ry. For the simple-cubic cell a = 10 bohr at Gamma with
|G|^2 < 20 Ry, the eigenvalues are (2 pi / a)^2 (m1^2 + m2^2 + m3^2) over
integer triples; the lowest 20 are written here, from integer arithmetic on
|m|^2 and one multiplication by (2 pi / a)^2.
"""
import itertools
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    a, ecut = 10.0, 20.0
    unit = (2.0 * math.pi / a) ** 2
    r = int(math.isqrt(int(ecut / unit))) + 1
    sq = sorted(m1 * m1 + m2 * m2 + m3 * m3 for m1, m2, m3 in itertools.product(range(-r, r + 1), repeat=3)
                if (m1 * m1 + m2 * m2 + m3 * m3) * unit < ecut)
    with open(os.path.join(HERE, "free_electron_c1.txt"), "w") as f:
        f.write("# lowest 20 free-electron eigenvalues (Ry), cubic a=10 bohr, Gamma: (2 pi/a)^2 |m|^2\n")
        for s in sq[:20]:
            f.write(f"{s * unit:.17e}\n")


if __name__ == "__main__":
    main()
