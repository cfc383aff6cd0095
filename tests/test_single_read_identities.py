"""CPU checks, with the oracle's c-transforms (eq. foc_f, foc_g) in FP64, of
the facts the single-read SK pass over a stored cost rests on:

1. For any pair (f, g), the column transform follows from the column sums
   M_j of the plan pi(f, g) (eq. Optimal_P_epsilon):
   T_c(f)_j = g_j - eps log(M_j / b_j).
2. With f = T_r(g), pi_ij = a_i t_ij / S_i for the row terms
   t_ij = b_j exp((g_j - C_ij - s_i)/eps) under any row shift s_i and their
   sum S_i = sum_j t_ij (the row-normalised plan).
3. With g = T_c(f_prev) and f = T_r(g): M_j >= b_j min_i a_i (any f_prev).
4. With the shift s_i = -f_prev_i: every t_ij <= b_j / a_i and S_i <= 1 / a_i;
   when f_prev is itself a row transform (every pass of the loop after a
   stage's first, which takes the max shift), also S_i >= min_j b_j.

None of this calls the library: it pins the algebra that the kernel and
its merge implement (Sec. 2, eq. SK_iterations)."""
import numpy as np
import pytest

import oracle as O


def _problem(n, m, seed, conc):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 2))
    y = rng.random((m, 2))
    C = O.sqeuclid_cost(x, y)
    a = rng.dirichlet(np.full(n, conc))
    b = rng.dirichlet(np.full(m, conc))
    return C, a, b, rng


CASES = [(40, 60, 1, 3.0, 5e-2), (70, 50, 2, 0.5, 2e-2), (30, 30, 3, 1.0, 1e-1), (55, 80, 4, 0.3, 3e-2)]


@pytest.mark.parametrize("n,m,seed,conc,eps", CASES)
def test_column_transform_from_plan_column_sums(n, m, seed, conc, eps):
    C, a, b, rng = _problem(n, m, seed, conc)
    f = rng.normal(0.0, 0.1, n)
    g = rng.normal(0.0, 0.1, m)
    M = O.coupling(f, g, C, a, b, eps).sum(axis=0)
    np.testing.assert_allclose(O.c_transform_col(f, C, a, eps), g - eps * np.log(M / b), rtol=0, atol=1e-12)


@pytest.mark.parametrize("n,m,seed,conc,eps", CASES)
def test_plan_is_row_normalised_terms(n, m, seed, conc, eps):
    C, a, b, rng = _problem(n, m, seed, conc)
    g = rng.normal(0.0, 0.1, m)
    f = O.c_transform_row(g, C, b, eps)
    P = O.coupling(f, g, C, a, b, eps)
    for shift in (np.zeros(n), rng.normal(0.0, 0.2, n), (g[None, :] - C).max(axis=1)):
        t = b[None, :] * np.exp((g[None, :] - C - shift[:, None]) / eps)
        S = t.sum(axis=1)
        np.testing.assert_allclose(a[:, None] * t / S[:, None], P, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n,m,seed,conc,eps", CASES)
def test_bounds_after_a_column_transform(n, m, seed, conc, eps):
    C, a, b, rng = _problem(n, m, seed, conc)
    # far from the optimum, so that the bounds are not trivially met
    for f_prev, row_transform in ((rng.normal(0.0, 0.3, n), False),
                                  (O.c_transform_row(rng.normal(0.0, 0.3, m), C, b, eps), True)):
        g = O.c_transform_col(f_prev, C, a, eps)
        f = O.c_transform_row(g, C, b, eps)
        M = O.coupling(f, g, C, a, b, eps).sum(axis=0)
        assert np.all(M >= b * a.min() * (1 - 1e-12))
        t = b[None, :] * np.exp((g[None, :] - C + f_prev[:, None]) / eps)
        assert np.all(t <= (b[None, :] / a[:, None]) * (1 + 1e-12))
        S = t.sum(axis=1)
        assert np.all(S <= (1.0 / a) * (1 + 1e-12))
        if row_transform:
            assert np.all(S >= b.min() * (1 - 1e-12))


def test_bounds_are_tight_enough_to_fail_on_a_wrong_shift():
    """A shift that drops f_prev (s = 0) breaks the term bound of check 4,
    and a random f_prev (not a row transform) breaks the lower bound of
    S_i: the bounds above are not vacuous."""
    C, a, b, rng = _problem(40, 60, 5, 1.0)
    eps = 2e-2
    f_prev = rng.normal(0.0, 0.3, 40) - 0.5
    g = O.c_transform_col(f_prev, C, a, eps)
    t = b[None, :] * np.exp((g[None, :] - C) / eps)
    assert np.any(t > b[None, :] / a[:, None])
    t = b[None, :] * np.exp((g[None, :] - C + f_prev[:, None]) / eps)
    assert np.any(t.sum(axis=1) < b.min())
