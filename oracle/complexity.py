"""The paper's multiplication-count model (Section 2.4).

TEST INFRASTRUCTURE (oracle).  Counts multiplications only, as Section 2.4
does; logarithms are base 2; the image is N^3, the detector N x N, and the
theoretical sampling N_rho = N, N_theta = N_phi = pi N (Section 2.4.1).

  FFT of length L: 0.5 L log L;  3D FFT: 1.5 N^3 log N (Section 2.4)
  step 1: C1a = 0.5 (16 N^3) log(16 N^3) + N^3 + 27 pi^2 N^3   (eq 2.16)
          C1b = pi^2 N^3                                        (eq 2.17)
          C1c = (pi N)^2 0.5 N log N                            (eq 2.18)
  step 2: C21 = two 16 N^3 FFTs + N^3 + 27 pi^2 N^3             (eq 2.19)
          C22 = 27 pi^2 N^3                                     (eq 2.20)
  step 3: C3a = pi^2 N^3, C3b = (pi N)^2 0.5 N log N,
          C3c = pi N ((2N)^2 log(2N) + (2N)^2 + 25 (2N)^2), C3d = pi N^3   (eq 2.21-2.24)
  CT projector: 8 N^3 pi N                                      (eq 2.27)
"""
from __future__ import annotations

import math

PI = math.pi


def lg(v: float) -> float:
    return math.log2(v)


def step1(N: float) -> dict:
    c1a = 0.5 * 16 * N ** 3 * lg(16 * N ** 3) + N ** 3 + 27 * PI ** 2 * N ** 3
    c1b = PI ** 2 * N ** 3
    c1c = (PI * N) ** 2 * 0.5 * N * lg(N)
    return {"C1a": c1a, "C1b": c1b, "C1c": c1c}


def step2(N: float) -> dict:
    c21 = 2 * (0.5 * 16 * N ** 3 * lg(16 * N ** 3)) + N ** 3 + 27 * PI ** 2 * N ** 3
    c22 = 27 * PI ** 2 * N ** 3
    return {"C21": c21, "C22": c22}


def step3(N: float) -> dict:
    c3a = PI ** 2 * N ** 3
    c3b = (PI * N) ** 2 * 0.5 * N * lg(N)
    c3c = PI * N * ((2 * N) ** 2 * lg(2 * N) + (2 * N) ** 2 + 25 * (2 * N) ** 2)
    c3d = PI * N * N ** 2
    return {"C3a": c3a, "C3b": c3b, "C3c": c3c, "C3d": c3d}


def total_method1(N: float) -> float:
    s1, s2, s3 = step1(N), step2(N), step3(N)
    return sum(s1.values()) + s2["C21"] + sum(s3.values())


def total_method2(N: float) -> float:
    s1, s2, s3 = step1(N), step2(N), step3(N)
    return sum(s1.values()) + s2["C22"] + sum(s3.values())


def ct_projector(N: float) -> float:
    return 8 * N ** 3 * PI * N


def fit_loglinear(fn, n1: float = 64.0, n2: float = 1024.0):
    """Coefficients (a, b) of fn(N)/N^3 = a log N + b from two sizes."""
    y1, y2 = fn(n1) / n1 ** 3, fn(n2) / n2 ** 3
    a = (y2 - y1) / (lg(n2) - lg(n1))
    return a, y1 - a * lg(n1)
