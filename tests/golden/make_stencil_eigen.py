"""Writes stencil_eigen.txt from the closed form of the 19-point sweep on a
separable sine mode (no implementation of the sweep is called).

With weights centre 1/4, face 1/16, edge 1/32 and the mode
p = sin(m pi i/(I-1)) sin(m pi j/(J-1)) sin(m pi k/(K-1)) (zero on the
boundary), each neighbour pair along axis d sums to 2 c_d p with
c_d = cos(m pi / (N_d - 1)), so one sweep multiplies the mode by
    mu = 1/4 + (c_x + c_y + c_z)/8 + (c_x c_y + c_y c_z + c_z c_x)/8.
The interior sum of p^2 is (I-1)(J-1)(K-1)/8, hence sweep n has residual
    r_n = (mu - 1)^2 mu^(2n-2) (I-1)(J-1)(K-1)/8.
"""
import math
import os

CASES = [(33, 33, 65, 1), (33, 33, 65, 4), (129, 129, 257, 1), (257, 257, 513, 1),
         (513, 513, 1025, 1), (19, 23, 71, 1), (19, 23, 71, 3)]


def mu(I, J, K, m):
    c = [math.cos(m * math.pi / (n - 1)) for n in (I, J, K)]
    return 0.25 + sum(c) / 8 + (c[0] * c[1] + c[1] * c[2] + c[2] * c[0]) / 8


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "stencil_eigen.txt")
    with open(path, "w") as f:
        f.write("# Closed form of the 19-point weighted-Jacobi sweep on the sine mode\n")
        f.write("# (written by make_stencil_eigen.py).  Columns: I J K m mu r_1 r_10\n")
        for I, J, K, m in CASES:
            u = mu(I, J, K, m)
            base = (I - 1) * (J - 1) * (K - 1) / 8.0
            r = [(u - 1) ** 2 * u ** (2 * n - 2) * base for n in (1, 10)]
            f.write("%d %d %d %d %.15e %.15e %.15e\n" % (I, J, K, m, u, r[0], r[1]))


if __name__ == "__main__":
    main()
