"""Systematic resampling with an exact integer CDF.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 (resampling) draws N particles from sum_n w_n delta_{v_n}; the paper does not
fix the scheme.  Systematic resampling is used: one uniform u in [0, 1) and the
points (i + u) / N, i = 0..N-1, each mapped to the first particle whose cumulative
weight exceeds it.  To make the result independent of summation order the CDF is
taken on integers:
    q_n = floor(W_n 2^53),  C_n = q_0 + ... + q_n,  Q = C_{N-1},
    p_i = floor((i 2^53 + u53) Q / (N 2^53)),   u53 = floor(u 2^53),
    idx_i = min{n : C_n > p_i}.
Python integers make every step exact.
"""
import bisect
import itertools
import math


def systematic(W, u53):
    N = len(W)
    q = [int(math.floor(float(w) * 2 ** 53)) for w in W]
    C = []
    run = 0
    for v in q:
        run += v
        C.append(run)
    Q = C[-1]
    if Q <= 0:
        raise ValueError("all weights are zero")
    D = N * 2 ** 53
    idx = []
    for i in range(N):
        p = ((i * 2 ** 53 + int(u53)) * Q) // D
        idx.append(bisect.bisect_right(C, p))      # first n with C_n > p
    return idx


def systematic_at(W, u53, outputs):
    """idx_i of systematic() for the listed outputs i only, by the same definition, for batches
    too large to list whole."""
    N = len(W)
    C = list(itertools.accumulate(int(math.floor(float(w) * 2 ** 53)) for w in W))
    Q = C[-1]
    if Q <= 0:
        raise ValueError("all weights are zero")
    D = N * 2 ** 53
    return [bisect.bisect_right(C, ((int(i) * 2 ** 53 + int(u53)) * Q) // D) for i in outputs]
