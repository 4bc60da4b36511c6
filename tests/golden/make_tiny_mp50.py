"""Writes tiny5_mp50.txt: a 5-body system and its accelerations, pair potential
and one vector-Jacobian product evaluated with mpmath at 50 significant digits.

The paper prints no worked numerical example (its validation compares against
a double-precision brute-force code, Sec. 4.1), so this fixture is brute force
at high precision instead: it is computed from the definitions directly, in
arbitrary precision, and does not call the oracle or the GPU library.

Definitions (Eq. (1) of Sec. 2.1 divided by m_i, Plummer softening of App. A):
  a_i  = G sum_{j != i} m_j d_ij / (|d_ij|^2 + eps^2)^(3/2),   d_ij = x_j - x_i
  W    = -G sum_{i < j} m_i m_j / (|d_ij|^2 + eps^2)^(1/2)
  phi  : phi_i = -G sum_{j != i} m_j / (|d_ij|^2 + eps^2)^(1/2), per particle
  VJP  : gx_k = sum_i (d a_i / d x_k)^T w_i,  gm_k = sum_i (d a_i / d m_k)^T w_i,
         obtained here by mpmath differentiation of the mpmath acceleration.
  jerk : d/dt a_i(x + V t) at t = 0 for velocities V (mpmath differentiation),
         the quantity App. A, Algorithm 3 accumulates beside the acceleration.
  snap : d^2/dt^2 a_i(x + V t + ACC t^2 / 2) at t = 0 for accelerations ACC
         (mpmath differentiation), the extra quantity a sixth-order Hermite
         step (Sec. 2.1) evaluates.
Run:  python tests/golden/make_tiny_mp50.py
"""
import os

import mpmath as mp

mp.mp.dps = 50

# Inputs are exact binary fractions so that float64 reads them without rounding.
X = [[0.5, -0.25, 0.125, 0.75, -0.625],
     [0.0, 0.375, -0.5, 0.25, 0.0625],
     [-0.125, 0.0, 0.25, -0.375, 0.5]]
M = [0.25, 0.125, 0.375, 0.0625, 0.1875]
G = 1.0
EPS = 0.0625
VEL = [[0.25, -0.5, 0.0, 0.125, -0.375],
       [0.5, 0.0, -0.25, 0.75, 0.0625],
       [-0.125, 0.375, 0.5, 0.0, -0.25]]
ACC = [[-0.5, 0.25, 0.125, -0.75, 0.375],
       [0.0625, -0.25, 0.5, 0.125, -0.5],
       [0.25, 0.0, -0.375, 0.5, 0.125]]
W_COT = [[0.5, -1.0, 0.25, 0.0, 0.75],
         [-0.5, 0.125, 1.0, -0.25, 0.0],
         [0.25, 0.5, -0.75, 1.0, -0.125]]


def accel(x, m, eps, G):
    n = len(m)
    out = [[mp.mpf(0)] * n for _ in range(3)]
    for i in range(n):
        for j in range(n):
            if j == i:
                continue
            d = [x[c][j] - x[c][i] for c in range(3)]
            s = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + eps ** 2
            f = G * m[j] / (s * mp.sqrt(s))
            for c in range(3):
                out[c][i] += f * d[c]
    return out


def potential(x, m, eps, G):
    n = len(m)
    w = mp.mpf(0)
    for i in range(n):
        for j in range(i + 1, n):
            d = [x[c][j] - x[c][i] for c in range(3)]
            w -= G * m[i] * m[j] / mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + eps ** 2)
    return w


def phi(x, m, eps, G):
    n = len(m)
    out = []
    for i in range(n):
        acc = mp.mpf(0)
        for j in range(n):
            if j != i:
                d = [x[c][j] - x[c][i] for c in range(3)]
                acc -= G * m[j] / mp.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2 + eps ** 2)
        out.append(acc)
    return out


def vjp(x, m, w, eps, G):
    """<w, a(x, m)> differentiated numerically at 50 digits (mpmath.diff)."""
    n = len(m)

    def contraction(xs, ms):
        a = accel(xs, ms, eps, G)
        return mp.fsum(w[c][i] * a[c][i] for c in range(3) for i in range(n))

    gx = [[mp.mpf(0)] * n for _ in range(3)]
    gm = [mp.mpf(0)] * n
    for c in range(3):
        for k in range(n):
            def f(t, c=c, k=k):
                xs = [[mp.mpf(v) for v in row] for row in x]
                xs[c][k] += t
                return contraction(xs, m)
            gx[c][k] = mp.diff(f, 0)
    for k in range(n):
        def g(t, k=k):
            ms = [mp.mpf(v) for v in m]
            ms[k] += t
            return contraction(x, ms)
        gm[k] = mp.diff(g, 0)
    return gx, gm


def jerk(x, vel, m, eps, G):
    """d/dt of the mpmath acceleration along straight-line motion x + vel t."""
    n = len(m)
    out = [[mp.mpf(0)] * n for _ in range(3)]
    for c in range(3):
        for i in range(n):
            def f(t, c=c, i=i):
                xs = [[x[d][k] + vel[d][k] * t for k in range(n)] for d in range(3)]
                return accel(xs, m, eps, G)[c][i]
            out[c][i] = mp.diff(f, 0)
    return out


def snap(x, vel, acc, m, eps, G):
    """d^2/dt^2 of the mpmath acceleration along x + vel t + acc t^2 / 2."""
    n = len(m)
    out = [[mp.mpf(0)] * n for _ in range(3)]
    for c in range(3):
        for i in range(n):
            def f(t, c=c, i=i):
                xs = [[x[d][k] + vel[d][k] * t + acc[d][k] * t * t / 2 for k in range(n)] for d in range(3)]
                return accel(xs, m, eps, G)[c][i]
            out[c][i] = mp.diff(f, 0, 2)
    return out


def main():
    x = [[mp.mpf(v) for v in row] for row in X]
    m = [mp.mpf(v) for v in M]
    w = [[mp.mpf(v) for v in row] for row in W_COT]
    eps, g = mp.mpf(EPS), mp.mpf(G)
    a = accel(x, m, eps, g)
    pot = potential(x, m, eps, g)
    ph = phi(x, m, eps, g)
    gx, gm = vjp(x, m, w, eps, g)
    vel = [[mp.mpf(v) for v in row] for row in VEL]
    jk = jerk(x, vel, m, eps, g)
    acc = [[mp.mpf(v) for v in row] for row in ACC]
    sn = snap(x, vel, acc, m, eps, g)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny5_mp50.txt")
    with open(path, "w") as f:
        f.write("# 5-body softened gravity evaluated with mpmath at 50 digits\n")
        f.write("# written by tests/golden/make_tiny_mp50.py; definitions in its docstring\n")
        f.write("# (Eq. (1) of Sec. 2.1 divided by m_i; softening of App. A as |d|^2+eps^2)\n")
        f.write("n 5\nG %r\neps %r\n" % (G, EPS))
        for c in range(3):
            f.write("x%d %s\n" % (c, " ".join(repr(v) for v in X[c])))
        f.write("m %s\n" % " ".join(repr(v) for v in M))
        for c in range(3):
            f.write("w%d %s\n" % (c, " ".join(repr(v) for v in W_COT[c])))
        for c in range(3):
            f.write("a%d %s\n" % (c, " ".join(mp.nstr(v, 40) for v in a[c])))
        f.write("W %s\n" % mp.nstr(pot, 40))
        for c in range(3):
            f.write("gx%d %s\n" % (c, " ".join(mp.nstr(v, 40) for v in gx[c])))
        f.write("gm %s\n" % " ".join(mp.nstr(v, 40) for v in gm))
        for c in range(3):
            f.write("v%d %s\n" % (c, " ".join(repr(v) for v in VEL[c])))
        for c in range(3):
            f.write("j%d %s\n" % (c, " ".join(mp.nstr(v, 40) for v in jk[c])))
        for c in range(3):
            f.write("acc%d %s\n" % (c, " ".join(repr(v) for v in ACC[c])))
        for c in range(3):
            f.write("s%d %s\n" % (c, " ".join(mp.nstr(v, 40) for v in sn[c])))
        f.write("phi %s\n" % " ".join(mp.nstr(v, 40) for v in ph))
    print("wrote", path)


if __name__ == "__main__":
    main()
