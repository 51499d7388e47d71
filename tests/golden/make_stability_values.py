"""Writes stability_values.json: closed forms of the two one-step methods on y' = lambda y.

Independent of the oracle and of the library (imports neither).  The coefficient tables are the
ones the paper prints: the Runge-Kutta-Fehlberg 4(5) tableau of Appendix B as exact rationals, and
the transformed ROS4 scheme of Appendix C (gamma = 0.57282 as tabulated, the a, c, m and E
columns to the printed 16 digits).  With z = h lambda and y0 = 1:

* RKF45: k_i = z (1 + sum_j a_ij k_j) is a polynomial in z; the propagated fourth-order solution
  is 1 + sum_j b_j k_j and the error estimate sum_j (bhat_j - b_j) k_j (exact rational arithmetic).
* ROS4: the stage equations (1/gamma - z) u_i = z (1 + sum_j a_ij u_j) + sum_j c_ij u_j are
  solved in turn at z = -1 and z = -1e12 in 40-digit arithmetic; R(z) = 1 + sum_i m_i u_i.

Run: python tests/golden/make_stability_values.py [--check]
"""
import json
import os
import sys
from fractions import Fraction as Fr

import mpmath

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "stability_values.json")

# Appendix B (Fehlberg): stage coefficients a_ij, fourth-order weights b, fifth-order weights bhat
RKF_A = [[],
         [Fr(1, 4)],
         [Fr(3, 32), Fr(9, 32)],
         [Fr(1932, 2197), Fr(-7200, 2197), Fr(7296, 2197)],
         [Fr(439, 216), Fr(-8), Fr(3680, 513), Fr(-845, 4104)],
         [Fr(-8, 27), Fr(2), Fr(-3544, 2565), Fr(1859, 4104), Fr(-11, 40)]]
RKF_B = [Fr(25, 216), Fr(0), Fr(1408, 2565), Fr(2197, 4104), Fr(-1, 5), Fr(0)]
RKF_BHAT = [Fr(16, 135), Fr(0), Fr(6656, 12825), Fr(28561, 56430), Fr(-9, 50), Fr(2, 55)]

# Appendix C (transformed ROS4 as printed; a4j = a3j, a43 = 0)
ROS_GAMMA = "0.57282"
ROS_A = [[], ["2.0"], ["1.867943637803922", "0.2344449711399156"],
         ["1.867943637803922", "0.2344449711399156", "0.0"]]
ROS_C = [[], ["-7.137615036412310"], ["2.580708087951457", "0.6515950076447975"],
         ["-2.137148994382534", "-0.3214669691237626", "-0.6949742501781779"]]
ROS_M = ["2.255570073418735", "0.2870493262186792", "0.4353179431840180", "1.093502252409163"]


def _padd(p, q):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]


def _pscale(p, s):
    return [s * c for c in p]


def rkf45_polys():
    """Stability polynomial of the propagated solution and of the error estimate (coefficients in z)."""
    k = []
    for i in range(6):
        arg = [Fr(1)]
        for j, a in enumerate(RKF_A[i]):
            arg = _padd(arg, _pscale(k[j], a))
        k.append([Fr(0)] + arg)                    # z * arg
    sol, err = [Fr(1)], [Fr(0)]
    for j in range(6):
        sol = _padd(sol, _pscale(k[j], RKF_B[j]))
        err = _padd(err, _pscale(k[j], RKF_BHAT[j] - RKF_B[j]))
    while sol and sol[-1] == 0:
        sol.pop()
    while err and err[-1] == 0:
        err.pop()
    return sol, err


def ros4_R(z):
    mpmath.mp.dps = 40
    z = mpmath.mpf(z)
    g = mpmath.mpf(ROS_GAMMA)
    u = []
    for i in range(4):
        rhs = z * (1 + sum(mpmath.mpf(a) * u[j] for j, a in enumerate(ROS_A[i])))
        rhs += sum(mpmath.mpf(c) * u[j] for j, c in enumerate(ROS_C[i]))
        u.append(rhs / (1 / g - z))
    return 1 + sum(mpmath.mpf(m) * ui for m, ui in zip(ROS_M, u))


def values():
    sol, err = rkf45_polys()
    zs = [-1.0, -1.0e12]
    return {
        "_source": "Closed forms of the methods' stability functions on y' = lambda*y, z = h*lambda, derived "
                   "from the coefficient tables the paper prints (Appendix B, Runge-Kutta-Fehlberg; Appendix C, "
                   "ROS4 with gamma = 0.57282) by exact rational / 40-digit arithmetic.  Written by "
                   "make_stability_values.py.",
        "rkf45_b_poly": {
            "_cite": "Appendix B: the fourth-order weights b reproduce exp(z) through z^4; their z^5 coefficient "
                     "is 1/104",
            "coeffs": [float(c) for c in sol]},
        "rkf45_err_poly": {
            "_cite": "Appendix B: sum_j (bhat_j - b_j) k_j on y' = lambda*y is (-z^5/780 + z^6/2080) y0",
            "coeffs": [float(c) for c in err]},
        "ros4_R": {
            "_cite": "Appendix C: ROS4 stability function R(z) (40-digit evaluation of the tabulated scheme); "
                     "R(-1e12) is the L-stable limit, small and negative",
            "z": zs,
            "R": [float(mpmath.nstr(ros4_R(z), 12)) for z in zs],
            "rel_tol": [1e-11, 1e-6]},
    }


if __name__ == "__main__":
    v = values()
    if "--check" in sys.argv:
        old = json.load(open(OUT))
        sys.exit(0 if old == v else 1)
    with open(OUT, "w") as fh:
        json.dump(v, fh, indent=2)
        fh.write("\n")
    print(OUT)
