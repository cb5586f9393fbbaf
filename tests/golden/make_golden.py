"""Writes the closed-form fixtures under tests/golden/.

Every value here comes from a closed form evaluated in 40-digit arithmetic
(mpmath); nothing is taken from the oracle or from the GPU library.

  chebyshev_n4.txt   Chebyshev points of the 2nd kind and barycentric weights
                     for n = 4 on [-1, 1] (eqs. 6-7): s_k = cos(pi k / 4),
                     w = (1/2, -1, 1, -1, 1/2).
  cube_corners.txt   Direct-sum potential (eq. 1, Coulomb and Yukawa kernels of
                     eq. 2) of 8 unit charges at the corners of the unit cube:
                     at each corner, 3 neighbours at distance 1, 3 at sqrt(2)
                     and 1 at sqrt(3), so phi = 3 G(1) + 3 G(sqrt 2) + G(sqrt 3).
  two_body.txt       Two charges q1, q2 at distance d: phi_1 = G(d) q2.
  regularized_two_body.txt
                     The same for the regularized Coulomb kernel
                     G(d) = (d^2 + delta^2)^(-1/2).

Run:  python tests/golden/make_golden.py
"""
import os

import mpmath as mp

mp.mp.dps = 40
HERE = os.path.dirname(os.path.abspath(__file__))


def g(r, kappa):
    return mp.e ** (-kappa * r) / r


def main():
    with open(os.path.join(HERE, "chebyshev_n4.txt"), "w") as f:
        f.write("# Chebyshev points of the 2nd kind, n = 4, [-1, 1] (eqs. 6-7)\n")
        f.write("# k s_k w_k\n")
        w = [mp.mpf(1) / 2, -1, 1, -1, mp.mpf(1) / 2]
        for k in range(5):
            f.write(f"{k} {mp.nstr(mp.chop(mp.cos(mp.pi * k / 4), tol=1e-30), 25)} {mp.nstr(mp.mpf(w[k]), 25)}\n")

    with open(os.path.join(HERE, "cube_corners.txt"), "w") as f:
        f.write("# 8 unit charges at the corners of [0,1]^3; potential at a corner (eq. 1)\n")
        f.write("# kappa phi   (kappa = 0 is the Coulomb kernel of eq. 2)\n")
        for kappa in (mp.mpf(0), mp.mpf("0.5"), mp.mpf(2)):
            phi = 3 * g(mp.mpf(1), kappa) + 3 * g(mp.sqrt(2), kappa) + g(mp.sqrt(3), kappa)
            f.write(f"{mp.nstr(kappa, 5)} {mp.nstr(phi, 25)}\n")

    with open(os.path.join(HERE, "two_body.txt"), "w") as f:
        f.write("# two charges at distance d: phi_1 = G(d) q2 (eqs. 1-2)\n")
        f.write("# d q2 kappa phi_1\n")
        for d, q2, kappa in (("0.125", "0.75", "0"), ("1.5", "-0.25", "0.5"), ("3", "1", "1.25")):
            d, q2, kappa = mp.mpf(d), mp.mpf(q2), mp.mpf(kappa)
            f.write(f"{mp.nstr(d, 10)} {mp.nstr(q2, 10)} {mp.nstr(kappa, 10)} "
                    f"{mp.nstr(g(d, kappa) * q2, 25)}\n")

    with open(os.path.join(HERE, "regularized_two_body.txt"), "w") as f:
        f.write("# two charges at distance d, G = (d^2 + delta^2)^(-1/2): phi_1 = G(d) q2\n")
        f.write("# d q2 delta phi_1\n")
        for d, q2, delta in (("0.125", "0.75", "0.01"), ("1.5", "-0.25", "0.5"), ("3", "1", "4")):
            d, q2, delta = mp.mpf(d), mp.mpf(q2), mp.mpf(delta)
            f.write(f"{mp.nstr(d, 10)} {mp.nstr(q2, 10)} {mp.nstr(delta, 10)} "
                    f"{mp.nstr(q2 / mp.sqrt(d * d + delta * delta), 25)}\n")


if __name__ == "__main__":
    main()
