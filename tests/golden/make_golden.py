"""Write ramp_exact.txt: exact solutions of the periodic heat stencil for the
paper's initial condition on small rings, in rational arithmetic.

Source of the values: Section 2 of the paper ("Model problem") -- the grid
x_i = i*h, the initial condition u(0, x) = x (here h = 1, so u0[i] = i), the
periodic boundary u(t, x) = u(t, L + x) and the explicit-Euler update of
Eq. (heat:discrete) with r = alpha*dt/h^2.  The solution after nt steps is
(I + r L)^nt u0 with L the circulant second difference, computed here in
exact fractions from that definition; nothing here calls the oracle or the
GPU library.  With integer data and r = 1/2 or 1/4 every value is a dyadic
rational with fewer than 53 significant bits, so binary64 evaluation in any
correct order reproduces these values exactly.

Run from the repository root: python tests/golden/make_golden.py
"""
import os
from fractions import Fraction

CASES = [(8, Fraction(1, 2), 12), (16, Fraction(1, 2), 12), (16, Fraction(1, 4), 12),
         (5, Fraction(1, 4), 9)]


def exact(N, r, nt):
    u = [Fraction(i) for i in range(N)]
    for _ in range(nt):
        u = [u[i] + r * (u[(i - 1) % N] - 2 * u[i] + u[(i + 1) % N]) for i in range(N)]
    return u


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "ramp_exact.txt"), "w") as f:
        f.write("# Exact solutions for the paper's ramp initial condition u0[i] = i (Section 2,\n"
                "# \"Model problem\": grid x_i = i*h with h = 1, u(0, x) = x, periodic boundary,\n"
                "# Eq. (heat:discrete) with r = alpha*dt/h^2), written by make_golden.py in exact\n"
                "# rational arithmetic.  One line per case: N r nt, then the N values as p/q.\n")
        for N, r, nt in CASES:
            u = exact(N, r, nt)
            f.write(f"{N} {r} {nt} " + " ".join(str(x) for x in u) + "\n")
    print("wrote", os.path.join(here, "ramp_exact.txt"))


if __name__ == "__main__":
    main()
