"""The KDE kernel's Gaussian terms on a uniform grid by the node-to-node
ratio recurrence (each lane holds 16 consecutive nodes), mirrored in float32
on the CPU and checked against direct float64 evaluation over the range
where the kernel uses it (node spacing S <= 1/4 in units of
h / sqrt(log2(e) / 2), and 2 S^2 (n_grid - 1) <= 64).

With x_i = x_0 + i S the term of sample k is 2^(-(x_i - x_k)^2) = u_i C_i,
u_0 = w_k 2^(-(x_0 - x_k)^2), u_i = u_{i-1} P, P = 2^(-2 S (x_0 - x_k)),
C_i = 2^(-(i S)^2) (by C_{i+1} = C_i r_i, r_i = 2^(-(2i+1) S^2),
r_{i+1} = r_i 2^(-2 S^2)); P is formed as 2^(-2 S x_0) 2^(2 S x_k).
"""
import numpy as np
import pytest

NB = 16
F = np.float32


def uses_recurrence(S, n_grid):
    return S <= 0.25 and 2.0 * S * S * (n_grid - 1) <= 64.0


def lane_terms_f32(x0l, S, zr, w):
    """sum_k w_k 2^(-(x_0 + i S - x_k)^2) for i < 16, as the kernel forms it."""
    S, x0l = F(S), F(x0l)
    r0 = np.exp2(F(-(S * S)))
    r2 = F(r0 * r0)
    C = np.empty(NB, F)
    ci, ri = F(1), r0
    for i in range(NB):
        C[i] = ci
        ci = F(ci * ri)
        ri = F(ri * r2)
    A = np.exp2(F(F(-2) * S * x0l))
    acc = np.zeros(NB, F)
    for z, wj in zip(np.asarray(zr, F), np.asarray(w, F)):
        P = F(A * np.exp2(F(F(2) * S * z)))
        x0 = F(x0l - z)
        u = F(wj * np.exp2(F(-(x0 * x0))))
        acc[0] = F(acc[0] + u)
        for i in range(1, NB):
            u = F(u * P)
            acc[i] = F(acc[i] + u)
    assert np.all(np.isfinite(acc))
    return (acc * C).astype(np.float64)


def lane_terms_direct(x0l, S, zr, w):
    x = x0l + S * np.arange(NB, dtype=np.float64)
    d = x[:, None] - np.asarray(zr, np.float64)[None, :]
    return (np.exp2(-d * d) * np.asarray(w, np.float64)[None, :]).sum(axis=1)


def check(x0l, S, zr, w):
    got = lane_terms_f32(x0l, S, zr, w)
    ref = lane_terms_direct(x0l, S, zr, w)
    tol = 1e-4 * ref + 1e-12 * max(ref.max(), np.max(w))
    assert np.all(np.abs(got - ref) <= tol), (x0l, S, np.max(np.abs(got - ref) / np.maximum(ref, 1e-300)))


@pytest.mark.parametrize("S", [0.01, 0.05, 0.1, 0.25])
def test_matches_direct_terms_on_a_256_node_grid(S):
    rng = np.random.default_rng(int(S * 1000))
    span = 255 * S
    zr = rng.uniform(0, span, 40)
    w = rng.lognormal(0.0, 1.0, 40)
    for lane in (0, 3, 8, 15):
        check(16 * lane * S, S, zr, w)


@pytest.mark.parametrize("S,n_grid", [(0.25, 256), (0.1768, 1024), (0.25, 513)])
def test_range_limits(S, n_grid):
    """At the edge of the range no factor leaves 2^(+-64): samples at both ends
    of the grid, lanes at both ends."""
    assert uses_recurrence(S, n_grid)
    span = (n_grid - 1) * S
    zr = np.array([0.0, 0.5 * S, span / 2, span - 0.5 * S, span])
    w = np.array([1.0, 3.0, 0.5, 2.0, 1.0])
    for x0l in (0.0, S * ((n_grid - 1) // 2), S * (n_grid - NB)):
        check(x0l, S, zr, w)
    assert (NB - 1) ** 2 * S * S <= 14.1           # u_i <= w_k 2^14
    assert 2 * S * span <= 64.0                    # 2^(-2 S x_0), 2^(2 S x_k) within 2^(+-64)


def test_outside_the_range():
    assert not uses_recurrence(0.26, 256)
    assert not uses_recurrence(0.2, 1024)           # 2 S^2 (n - 1) = 81.8
    assert uses_recurrence(0.25, 256)


def test_samples_outside_the_support_add_exact_zeros():
    """Samples beyond the redshift support carry w = 0 and x_k far below the
    grid: their factor underflows to 0 and adds nothing (no NaN)."""
    S = 0.05
    zr = np.array([-5000.0, 3.0])
    w = np.array([0.0, 1.0])
    got = lane_terms_f32(0.0, S, zr, w)
    ref = lane_terms_direct(0.0, S, zr[1:], w[1:])
    assert np.all(np.abs(got - ref) <= 1e-4 * ref + 1e-30)
