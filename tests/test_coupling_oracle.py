"""Pins of the TO-coupling oracle (Sec. 2.2: Eqs. Heaviside, accFilter,
filtered_sens) against closed forms, limits and hand-checked cases."""
import math

import numpy as np

from oracle import coupling as cp


def test_heaviside_end_points_and_grid():
    for beta in (0.5, 2.0, 8.0, 30.0):
        r = cp.heaviside([0.0, 1.0, -0.3, 1.7], beta)
        assert r.tolist() == [0.0, 1.0, 0.0, 1.0]      # rho(0) = 0, rho(1) = 1, clamped
    x = np.linspace(0, 1, 10001)
    r = cp.heaviside(x, 8.0).astype(np.float64)
    assert np.array_equal(r * 2 ** 24, np.round(r * 2 ** 24))   # on the 2^-24 grid
    assert (np.diff(r) >= 0).all()                              # monotone for beta > 0


def test_heaviside_limits():
    x = np.linspace(0, 1, 1001)
    # beta -> 0: 1 - e^{-b x} + x e^{-b} = x + O(b)  (identity projection)
    r = cp.heaviside(x, 1e-9).astype(np.float64)
    assert np.abs(r - x).max() <= 2 ** -24
    # beta large: a step; with beta = 60 every x >= 0.3 has 1 - rho = e^{-60 x}
    # (1 - x) < 2^-25 and rounds to 1, and x = 0.01 gives 1 - e^{-0.6} (+ ~0)
    r = cp.heaviside(x[300:], 60.0).astype(np.float64)
    assert (r == 1.0).all()
    assert abs(float(cp.heaviside([0.01], 60.0)[0]) - (1 - math.exp(-0.6))) < 2 ** -24
    # slope at 0 is beta + e^{-beta}
    b = 2.0
    h = 1e-3
    slope = float(cp.heaviside([h], b)[0]) / h
    assert abs(slope - (b + math.exp(-b))) < 2e-3 * b


def test_access_filter_cases():
    design = np.array([0.2, 0.7, 0.4, 0.9, 0.5], np.float32)
    fbar = np.array([0.3, 0.6, 0.8, 0.0, 0.9], np.float32)
    sec = np.array([0, 0, 1, 0, 1], np.uint8)
    f = cp.access_filter(design, fbar, sec, tau=0.5)
    # void not secluded -> 0; solid -> fbar; secluded void -> 1; solid with
    # fbar 0 -> 0; rho == tau is void -> secluded -> 1
    assert f.tolist() == [0.0, np.float32(0.6), 1.0, 0.0, 1.0]


def test_filtered_sensitivity_is_a_convex_combination():
    rng = np.random.default_rng(3)
    s = rng.normal(size=1000).astype(np.float32)
    filt = rng.random(1000).astype(np.float32)
    om = rng.random(1000) < 0.8
    m = np.abs(s[om]).max()
    out = cp.filtered_sensitivity(s, filt, 0.0, om)
    assert np.allclose(out, s / m, rtol=0, atol=1e-7)
    assert np.abs(out[om]).max() == np.float32(1.0)
    out = cp.filtered_sensitivity(s, filt, 1.0, om)
    assert np.array_equal(out, filt)
    w = 0.3
    out = cp.filtered_sensitivity(s, filt, w, om).astype(np.float64)
    assert np.allclose(out, (1 - w) * s / m + w * filt, atol=1e-7)
    assert np.array_equal(cp.filtered_sensitivity(np.zeros(5), np.ones(5), 0.5,
                                                  np.ones(5, bool)), np.full(5, 0.5, np.float32))


def test_greedy_plan_hand_case():
    # 1D negative space of 10 voxels (design 0), three orientations
    design = np.zeros(10)
    design[[0, 9]] = 1                       # solid at both ends: N = voxels 1..8
    A = np.zeros((3, 10), bool)
    A[0, 1:4] = True                          # covers 3
    A[1, 3:9] = True                          # covers 6 (largest)
    A[2, 1:3] = True                          # covers 2, then 2 after step 1
    steps, left = cp.plan_greedy(A, design)
    assert steps == [(1, 6), (0, 2)] and left == 0
    # ties go to the lowest index; unreachable voxels remain
    A2 = np.zeros((2, 10), bool)
    A2[0, 1:3] = A2[1, 5:7] = True
    steps, left = cp.plan_greedy(A2, design)
    assert steps == [(0, 2), (1, 2)] and left == 4
    assert cp.plan_greedy(A2, design, max_steps=1) == ([(0, 2)], 6)


def test_greedy_plan_invariants():
    rng = np.random.default_rng(11)
    A = rng.random((9, 500)) < 0.2
    design = (rng.random(500) < 0.3).astype(np.float32)
    om = rng.random(500) < 0.9
    steps, left = cp.plan_greedy(A, design, omega0=om)
    N = om & (design <= 0.5)
    # what is left is exactly the negative space no orientation reaches
    assert left == int(np.count_nonzero(N & ~A.any(0)))
    # the removed counts sum to the reachable part and never increase
    assert sum(r for _, r in steps) == int(np.count_nonzero(N & A.any(0)))
    assert all(steps[i][1] >= steps[i + 1][1] for i in range(len(steps) - 1))


def test_filtered_sensitivity_hand_case_intermediate_weight():
    """Eq. filtered_sens at w = 0.35 on five values worked by hand: the
    normalization is the largest |S_phi| over Omega_0 only (element 3, outside
    Omega_0, holds the global largest, 8, and is not used: the divisor is 4);
    Sbar = [0.5, -1, 0.25, 2, -0.75]; the result is 0.65 Sbar + 0.35 filter."""
    s = np.array([2.0, -4.0, 1.0, 8.0, -3.0], np.float32)
    filt = np.array([0.2, 1.0, 0.0, 0.5, 0.8], np.float32)
    om = np.array([1, 1, 1, 0, 1], bool)
    out = cp.filtered_sensitivity(s, filt, 0.35, om)
    expect = [0.395, -0.3, 0.1625, 1.475, -0.2075]
    assert out.dtype == np.float32
    assert out.tolist() == [float(np.float32(v)) for v in expect]
