#!/usr/bin/env python3
"""Minimax polynomial coefficients for the FP32 device operators (fp32_math.h).

A Remez exchange in FP64 (numpy): for a target g(u) on [a, b] and a weight
w(u) it finds the polynomial p of degree n that minimises
max |(p(u) - g(u)) w(u)|, by solving for n + 2 alternating reference points,
moving them to the extrema of the weighted error and repeating until the
error levels off.  The coefficients are then rounded to FP32, and the error
of the rounded polynomial is measured on a dense grid (the device evaluates
it in FP32 with fused multiply-adds; the host checks in tests/ measure the
whole operator against the C library).

    sinpi:  sin(pi t) = t S(t^2),          t in [0, 1/4], S of degree 3
    cospi:  cos(pi t) = 1 + t^2 C(t^2),    t in [0, 1/4], C of degree 3
            (both weighted to relative error; |t| <= 1/4 after the exact
            quarter-period reduction)
    exp2:   2^f = 1 + f E(f),              f in [-1/2, 1/2], E of degree 6
            (relative error)

Run:  python gen_minimax.py     prints the FP32 coefficients and errors
"""
import numpy as np


def remez(g, w, a, b, n, iters=60, grid=20001):
    """Weighted minimax polynomial of degree n for g on [a, b]; returns the
    FP64 coefficients (lowest degree first) and the levelled error."""
    k = np.arange(n + 2)
    x = 0.5 * (a + b) + 0.5 * (b - a) * -np.cos(np.pi * k / (n + 1))  # Chebyshev extrema
    us = np.linspace(a, b, grid)
    E = 0.0
    for _ in range(iters):
        A = np.zeros((n + 2, n + 2))
        for i in range(n + 2):
            A[i, :n + 1] = x[i] ** np.arange(n + 1)
            A[i, n + 1] = (-1) ** i / w(x[i])
        sol = np.linalg.solve(A, g(x))
        c, E = sol[:n + 1], sol[n + 1]
        err = (np.polyval(c[::-1], us) - g(us)) * w(us)
        # new reference: the extremum of each run of one error sign
        sgn = np.sign(err)
        runs = np.split(np.arange(grid), np.nonzero(np.diff(sgn) != 0)[0] + 1)
        ext = [r[np.argmax(np.abs(err[r]))] for r in runs if len(r)]
        if len(ext) < n + 2:
            break
        # keep n + 2 alternating extrema with the largest error
        while len(ext) > n + 2:
            if abs(err[ext[0]]) < abs(err[ext[-1]]):
                ext = ext[1:]
            else:
                ext = ext[:-1]
        nx = us[ext]
        if np.allclose(nx, x, rtol=0, atol=1e-15):
            break
        x = nx
    return c, abs(E)


def f32(c):
    return np.asarray(c, np.float32)


def horner32(c, u):
    """FP32 Horner with fused multiply-adds (FP64 product of FP32 values is
    exact; the sum is rounded once to FP32 as the device's fma rounds)."""
    u = np.asarray(u, np.float32).astype(np.float64)
    r = np.full(u.shape, np.float64(np.float32(c[-1])))
    for ck in c[-2::-1]:
        r = np.float32(r * u + np.float64(np.float32(ck))).astype(np.float64)
    return r


def sinpi_coeffs():
    g = lambda z: np.where(z == 0, np.pi, np.sin(np.pi * np.sqrt(z)) / np.sqrt(np.where(z == 0, 1, z)))
    c, e = remez(g, lambda z: 1.0 / g(z), 0.0, 1.0 / 16.0, 3)
    return c, e


def cospi_coeffs():
    # cos(pi t) = 1 + z C(z): fit C = (cos(pi sqrt z) - 1) / z, weighted so
    # that the error of 1 + z C is relative to cos(pi t)
    def g(z):
        zz = np.where(z == 0, 1.0, z)
        return np.where(z == 0, -np.pi ** 2 / 2, (np.cos(np.pi * np.sqrt(zz)) - 1.0) / zz)
    w = lambda z: np.maximum(z, 1e-300) / np.cos(np.pi * np.sqrt(z))
    c, e = remez(g, w, 1e-12, 1.0 / 16.0, 3)
    return c, e


def exp2_coeffs():
    def g(f):
        ff = np.where(f == 0, 1.0, f)
        return np.where(f == 0, np.log(2.0), np.expm1(np.log(2.0) * ff) / ff)
    w = lambda f: np.abs(np.where(f == 0, 1e-300, f)) / np.exp2(f)
    c, e = remez(g, w, -0.5, 0.5, 6)
    return c, e


def main():
    z = np.linspace(0, 1 / 16, 200001)
    t = np.sqrt(z)
    c, e = sinpi_coeffs()
    got = np.sqrt(z) * horner32(f32(c), z)
    ref = np.sin(np.pi * t)
    m = t > 0
    print("sinpi S (degree 3): levelled relative error %.3g" % e)
    print("  FP32:", ", ".join("%.9e" % v for v in f32(c)))
    print("  FP32 Horner max relative error %.3g" % np.max(np.abs(got[m] - ref[m]) / ref[m]))
    c, e = cospi_coeffs()
    got = 1.0 + z * horner32(f32(c), z)
    ref = np.cos(np.pi * t)
    print("cospi C (degree 3): levelled relative error %.3g" % e)
    print("  FP32:", ", ".join("%.9e" % v for v in f32(c)))
    print("  max relative error %.3g" % np.max(np.abs(got - ref) / ref))
    c, e = exp2_coeffs()
    f = np.linspace(-0.5, 0.5, 200001)
    got = 1.0 + f * horner32(f32(c), f)
    print("exp2 E (degree 6): levelled relative error %.3g" % e)
    print("  FP32:", ", ".join("%.9e" % v for v in f32(c)))
    print("  max relative error %.3g" % np.max(np.abs(got - np.exp2(f)) / np.exp2(f)))


if __name__ == "__main__":
    main()
