"""Writes steady_slab_n16.txt: the oracle's converged solution of the steady
1-D heat-transfer problem (Sec. 5.3.2, the Fourier flow; Appendix B scheme) on a
small grid, for the GPU solver's parity test.  Calls only oracle/ and the
input generators.

    python tests/golden/make_steady.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import quadrature, steady  # noqa: E402

CFG = dict(n=16, L=5.0, omega=0.74, nx=4, kn=0.1, theta_l=1.0, theta_r=1.5, mass=1.0, tol=1e-10)
SAMPLES = 48


def main():
    c = CFG
    P = steady.Problem(c["n"], c["L"], c["omega"], c["nx"], c["kn"], c["theta_l"], c["theta_r"],
                       mass=c["mass"], sphere=quadrature.hemisphere_product_rule(8, 16))
    f, hist = P.solve(tol=c["tol"], max_newton=30)
    mom = P.moments(f)
    rng = np.random.default_rng(2025)
    idx = np.stack([rng.integers(0, c["nx"], SAMPLES)] + [rng.integers(0, c["n"], SAMPLES) for _ in range(3)], 1)
    out = os.path.join(HERE, "steady_slab_n16.txt")
    with open(out, "w") as fh:
        fh.write("# Oracle solution of the steady 1-D heat-transfer problem (Sec. 5.3.2; scheme of\n")
        fh.write("# Appendix B; readings: zero-flux wall densities, Q with Q^_0 = 0, P L P in the\n")
        fh.write("# Newton operator, iterates rescaled to the mass C).  Written by\n")
        fh.write("# tests/golden/make_steady.py from oracle/ only.\n")
        fh.write("# config " + " ".join(f"{k}={v}" for k, v in c.items()) + "\n")
        fh.write("# hemisphere rule: 8-point Gauss-Legendre (4 positive cosines) x 16 azimuths\n")
        fh.write("# residual history " + " ".join(f"{h:.6e}" for h in hist) + "\n")
        fh.write(f"# mass {P.total_mass(f):.17e}\n")
        fh.write("# moments: cell rho u1 u2 u3 theta\n")
        for j in range(c["nx"]):
            fh.write("M %d " % j + " ".join(f"{v:.17e}" for v in mom[j]) + "\n")
        fh.write("# samples: cell i1 i2 i3 f\n")
        for a, b, d, e in idx:
            fh.write(f"F {a} {b} {d} {e} {f[a, b, d, e]:.17e}\n")
    print(out, hist)


if __name__ == "__main__":
    main()
