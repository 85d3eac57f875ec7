"""The identity behind the specialised 2D SG operator, checked on the CPU with the
oracle's quadrature moments (no GPU code involved).

The operator evaluates the k² block E[k² φ_i φ_j] (eq. c_ij) as K_extᵀ K_ext with
K_ext[m, j] = E[k φ_m φ_j] over the multi-indices m of total degree <= r+1, and the
boundary block E[k φ_i φ_j] (eq. b_ij) as the leading part of the same K.  K is the
three-term Legendre recurrence per variable, ξ φ_a = β_{a+1} φ_{a+1} + β_a φ_{a-1} with
β_a = a / sqrt(4a² - 1), and in the unknowns scaled by ν_j = Π_l β_1⋯β_{j_l} its
entries towards lower degree are k_l and towards higher degree k_l β².
"""
import math

import numpy as np
import pytest

from oracle import pc


def beta(a):
    return a / math.sqrt(4.0 * a * a - 1.0)


@pytest.mark.parametrize("s,r", [(1, 3), (2, 2), (3, 3), (4, 3), (6, 3)])
def test_k2_block_factorises_through_degree_r_plus_1(s, r):
    rng = np.random.default_rng(s * 10 + r)
    k = np.concatenate([[rng.uniform(5.0, 20.0)], rng.uniform(-2.0, 2.0, s)])   # k_0, k_1..k_s at one point
    E = pc.moment_tables(s, r)
    Eext = pc.moment_tables(s, r + 1)
    Q = pc.basis_size(s, r)
    # the degree <= r basis is the leading part of the degree <= r+1 basis (graded order)
    np.testing.assert_array_equal(pc.multi_indices(s, r + 1)[:Q], pc.multi_indices(s, r))
    C = sum(k[a] * k[b] * E[a, b] for a in range(s + 1) for b in range(s + 1))
    Kext = sum(k[a] * Eext[a, 0] for a in range(s + 1))[:, :Q]
    np.testing.assert_allclose(Kext.T @ Kext, C, rtol=0, atol=1e-12 * np.abs(C).max())
    # the boundary block is K restricted to the basis
    B = sum(k[a] * E[a, 0] for a in range(s + 1))
    np.testing.assert_allclose(Kext[:Q], B, rtol=0, atol=1e-13 * np.abs(B).max())


@pytest.mark.parametrize("s,r", [(2, 3), (4, 3), (6, 3)])
def test_k_factor_is_the_scaled_three_term_recurrence(s, r):
    rng = np.random.default_rng(7)
    k = np.concatenate([[rng.uniform(5.0, 20.0)], rng.uniform(-2.0, 2.0, s)])
    alpha = pc.multi_indices(s, r + 1)
    Q = pc.basis_size(s, r)
    Kext = sum(k[a] * pc.moment_tables(s, r + 1)[a, 0] for a in range(s + 1))[:, :Q]
    nu = np.array([np.prod([beta(b) for l in range(s) for b in range(1, a[l] + 1)]) for a in alpha])
    scaled = Kext * nu[None, :Q] / nu[:, None]
    index = {tuple(a): q for q, a in enumerate(alpha)}
    expect = np.zeros_like(scaled)
    for j in range(Q):
        expect[j, j] = k[0]
        for l in range(s):
            a = list(alpha[j])
            a[l] += 1
            expect[index[tuple(a)], j] = k[l + 1]                          # row of higher degree: weight k_l
            if alpha[j][l] > 0:
                a[l] -= 2
                expect[index[tuple(a)], j] = k[l + 1] * beta(alpha[j][l]) ** 2   # lower degree: k_l β²
    np.testing.assert_allclose(scaled, expect, rtol=0, atol=1e-12 * abs(k).max())
