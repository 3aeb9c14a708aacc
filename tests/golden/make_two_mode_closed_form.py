"""Writes two_mode_closed_form.json: J and dJ/dA of the periodic two-amplitude
identification (reading C10: body force A1 b1 + A2 b2, target the continuum
displacement of A* = (0.7, 0.3), E = 1, nu = 0.3) at A = (0.1, 0.1), from the
closed-form fixed point of the scheme (oracle/fourier.py: one 8 x 8 solve per
wavevector, eq. primal_fixed_point) and the objective of eq. node_J with C-bar
in closed form.

C-bar = sum_n |d*_n|^2 dx^2 with d* = c1 b1 + c2 b2, c1 = A1*/(8 pi^2 (mu+K)),
c2 = A2*/(16 pi^2 (mu+K)): by discrete orthogonality of the sampled sines and
cosines (N >= 5), sum |b1|^2 = N^2/2, sum |b2|^2 = N^2, sum b1.b2 = 0, and
N^2 dx^2 = 1, so C-bar = c1^2 / 2 + c2^2.

Run from the repository root:  python tests/golden/make_two_mode_closed_form.py
Calls only oracle/ and the seeded input generators.
"""
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fourier as Fo  # noqa: E402
from paper_2609_31347_amd import inputs as I  # noqa: E402


def closed_form(n, a=(0.1, 0.1), E=1.0, nu=0.3, A_star=(0.7, 0.3)):
    s = E / (1.0 - nu * nu)                     # mu + K
    c1 = A_star[0] / (8 * math.pi ** 2 * s)
    c2 = A_star[1] / (16 * math.pi ** 2 * s)
    cbar = 0.5 * c1 * c1 + c2 * c2
    modes = I.two_mode_basis(n)
    tgt = I.two_mode_target(n, E, nu, A_star)
    dx2 = 1.0 / n ** 2
    H = Fo.transfer(n, n, E, nu)
    d = Fo.steady_disp(dx2 * np.tensordot(np.asarray(a), modes, 1), E, nu, H)
    r = d - tgt
    J = 0.5 * float((r ** 2).sum()) * dx2 / cbar
    gg = Fo.grad_g(r, E, nu, H) * dx2 / cbar
    grad = [float((gg * dx2 * m).sum()) for m in modes]
    return {"n": n, "A": list(a), "E": E, "nu": nu, "A_star": list(A_star), "cbar": cbar, "J": J,
            "grad": grad}


def main():
    out = {"_about": "Closed-form J and dJ/dA of the periodic two-amplitude identification "
                     "(reading C10; eq. node_J with C-bar in closed form; eq. optimality), written by "
                     "tests/golden/make_two_mode_closed_form.py from the Fourier fixed point of the scheme "
                     "(eq. primal_fixed_point per wavevector).",
           "cases": [closed_form(16), closed_form(32)]}
    path = os.path.join(HERE, "two_mode_closed_form.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(path)


if __name__ == "__main__":
    main()
