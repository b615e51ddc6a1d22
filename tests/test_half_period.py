"""The half-period identities the GPU synthesis relies on, checked on the CPU.

The kernels evaluate the grid sums of u~ = Phi^T x^ (N = 4K points
xi_j = -pi + 2 pi j/N) from the even-mode and odd-mode syntheses E_j, O_j on
the first half of the grid only: shifting xi by pi multiplies mode k by
(-1)^k, so u~_j = E_j + O_j and u~_{j+N/2} = E_j - O_j, and

    sum_j u~_j   = sum_{j<N/2} 2 E_j
    sum_j u~_j^2 = sum_{j<N/2} 2 (E_j^2 + O_j^2)
    sum_j u~_j^3 = sum_{j<N/2} 2 E_j (E_j^2 + 3 O_j^2)
    sum_j u~_j^4 = sum_{j<N/2} 2 ((E_j^2 + O_j^2)^2 + 4 E_j^2 O_j^2).

The cube sum is also checked in the form the kernels evaluate it, from odd-mode
syntheses whose rows carry the factor sqrt(3): 2 E (E^2 + o^2), o = sqrt(3) O.
Likewise the mixture's Woodbury term y^T G^-1 y as |C y|^2 with the Cholesky
factor C the y tables carry.

Here E and O are formed directly from their definitions (cos/sin sums over
the modes of one parity) and compared with the oracle's grid (`oracle.grid`,
the full synthesis on all N points), in FP64.  The pair-term bound the decision
window uses, 2 |E| (E^2 + 3 O^2) <= |u~_j|^3 + |u~_{j+N/2}|^3, is checked too,
and the mode order of the operand split (entry e of k-step s: modes
16 s + 2 e + 2 for the even part, 16 s + 2 e + 1 for the odd part) against the
gather of the plain fragments (odd entries of k-steps 2s and 2s + 1).
"""
import math

import numpy as np
import pytest

import oracle


def _parity_syntheses(x, K, N):
    """E_j, O_j for j < N/2 from x = [cos block | sin block] (unscaled)."""
    j = np.arange(N // 2)
    xi = -math.pi + 2 * math.pi * j / N
    E = np.zeros(N // 2)
    O = np.zeros(N // 2)
    for k in range(1, K + 1):
        term = x[k - 1] * np.cos(k * xi) + x[K + k - 1] * np.sin(k * xi)
        if k % 2 == 0:
            E += term
        else:
            O += term
    return E, O


@pytest.mark.parametrize("K", [16, 32, 64])
def test_power_sums_from_half_the_grid(K):
    N = 4 * K
    rng = np.random.default_rng(K)
    amp = math.sqrt(2.0 / math.pi)  # E0 = 1: the oracle's u = amp u~
    for _ in range(20):
        x = rng.standard_normal(2 * K) / np.sqrt(1.0 + np.tile(np.arange(K), 2))
        x /= np.linalg.norm(x)
        u = oracle.grid(x, 1.0, N) / amp
        E, O = _parity_syntheses(x, K, N)
        # the two halves of the grid
        assert np.allclose(u[: N // 2], E + O, atol=1e-13)
        assert np.allclose(u[N // 2:], E - O, atol=1e-13)
        scale = np.sum(np.abs(u) ** 4) + 1.0
        assert abs(np.sum(u) - np.sum(2 * E)) < 1e-12 * scale
        assert abs(np.sum(u ** 2) - np.sum(2 * (E * E + O * O))) < 1e-12 * scale
        assert abs(np.sum(u ** 3) - np.sum(2 * E * (E * E + 3 * O * O))) < 1e-12 * scale
        w = E * E + O * O
        assert abs(np.sum(u ** 4) - np.sum(2 * (w * w + 4 * E * E * O * O))) < 1e-12 * scale
        # the cube kernels read odd-mode rows scaled by sqrt(3): o = sqrt(3) O
        o = math.sqrt(3.0) * O
        assert abs(np.sum(u ** 3) - np.sum(2 * E * (E * E + o * o))) < 1e-12 * scale
        # Parseval on the grid (|x^| = 1): sum u~^2 = N/2, and sum u~ = 0
        assert abs(np.sum(u ** 2) - N / 2) < 1e-10
        assert abs(np.sum(u)) < 1e-10
        # the bound used by the decision window, pair by pair
        lhs = 2 * np.abs(E) * (E * E + 3 * O * O)
        rhs = np.abs(E + O) ** 3 + np.abs(E - O) ** 3
        assert np.all(lhs <= rhs * (1 + 1e-12) + 1e-15)


def test_the_split_needs_only_an_even_grid():
    # N = 3K is below the exactness threshold N > 3K of the cube quadrature;
    # the half-period split itself still holds (it only needs N even)
    K = 16
    N = 3 * K
    rng = np.random.default_rng(5)
    x = rng.standard_normal(2 * K)
    x /= np.linalg.norm(x)
    u = oracle.grid(x, 1.0, N) / math.sqrt(2.0 / math.pi)
    E, O = _parity_syntheses(x, K, N)
    assert np.allclose(u[: N // 2], E + O, atol=1e-13)


@pytest.mark.parametrize("K", [16, 32, 64])
def test_parity_operand_order_matches_the_table_gather(K):
    # plain fragment (k-step s) entry e holds mode 8 s + e + 1; the gather
    # takes entries 1, 3, 5, 7 (even modes) or 0, 2, 4, 6 (odd modes) of
    # k-steps 2s and 2s + 1
    for s in range(K // 16):
        for p in (0, 1):
            gathered = [8 * (2 * s + e // 4) + 2 * (e % 4) + (1 - p) + 1 for e in range(8)]
            operand = [16 * s + 2 * e + 2 - p for e in range(8)]
            assert gathered == operand
    # together the parities cover every mode once
    modes = sorted(16 * s + 2 * e + 2 - p for s in range(K // 16) for p in (0, 1) for e in range(8))
    assert modes == list(range(1, K + 1))


def test_folded_cholesky_factor_gives_the_woodbury_term():
    # the mixture's y tables carry C with C^T C = G^-1 (c00 = sqrt(m00),
    # c01 = m01/c00, c11 = sqrt(m11 - c01^2)), so |C y|^2 = y^T G^-1 y; and
    # |C|_2 <= 1 whenever G >= I, which keeps the window's product term valid
    rng = np.random.default_rng(3)
    for _ in range(200):
        B = rng.standard_normal((2, 2)) * rng.uniform(0.01, 10.0)
        G = np.eye(2) + B @ B.T  # I + V^T D^-1 V is of this form
        M = np.linalg.inv(G)
        c00 = math.sqrt(M[0, 0])
        c01 = M[0, 1] / c00
        c11 = math.sqrt(max(0.0, M[1, 1] - c01 * c01))
        C = np.array([[c00, c01], [0.0, c11]])
        assert np.allclose(C.T @ C, M, rtol=1e-12, atol=1e-15)
        y = rng.standard_normal(2)
        assert abs(np.sum((C @ y) ** 2) - y @ M @ y) <= 1e-12 * (y @ M @ y + 1e-300) + 1e-15
        assert np.linalg.norm(C, 2) <= 1.0 + 1e-12


# --------------------------------------------------------------------------
# Quarter-period form (K = 128): cos/sin blocks and mode parities separately
# --------------------------------------------------------------------------

def _quarter_syntheses(x, K, N):
    """Ce, Co, Se, So on the representatives xi_j = -pi + 2 pi (j + 1/2)/N with
    xi in (0, pi/2) (j = N/2 .. 3N/4 - 1): cos/sin block times even/odd modes."""
    j = np.arange(N // 2, 3 * N // 4)
    xi = -math.pi + 2 * math.pi * (j + 0.5) / N
    k = np.arange(1, K + 1)
    C, S = np.cos(np.outer(xi, k)), np.sin(np.outer(xi, k))
    ev = k % 2 == 0
    return (C[:, ev] @ x[:K][ev], C[:, ~ev] @ x[:K][~ev], S[:, ev] @ x[K:][ev], S[:, ~ev] @ x[K:][~ev])


@pytest.mark.parametrize("K", [32, 128])
def test_cube_sum_from_a_quarter_of_the_offset_grid(K):
    """On the grid offset by half a step, xi -> -xi and xi -> xi + pi map the
    representatives in (0, pi/2) onto the other three quadrants, where
    u~ = (Ce + Co) +- (Se + So) and (Ce - Co) +- (Se - So); the four cubes sum to
    4 Ce (Ce^2 + 3 Co^2 + 3 Se^2 + 3 So^2) + 24 Co Se So, and the trapezoid sum
    of u^3 on any equispaced grid with N >= 3K + 1 points is (3N/pi) times H3
    (the definition of H3 as (1/6) int u^3), so it equals the standard grid's
    sum.  The kernels read the Co, Se, So rows times sqrt(3):
    4 Ce (Ce^2 + co^2 + se^2 + so^2) + (8/sqrt 3) co se so."""
    N = 4 * K
    rng = np.random.default_rng(K + 1)
    amp = math.sqrt(2.0 / math.pi)
    r3 = math.sqrt(3.0)
    for _ in range(10):
        x = rng.standard_normal(2 * K) / np.sqrt(1.0 + np.tile(np.arange(K), 2))
        x /= np.linalg.norm(x)
        u = oracle.grid(x, 1.0, N) / amp
        ref, scale = np.sum(u ** 3), np.sum(np.abs(u) ** 3)
        Ce, Co, Se, So = _quarter_syntheses(x, K, N)
        s3 = np.sum(4 * Ce * (Ce ** 2 + 3 * Co ** 2 + 3 * Se ** 2 + 3 * So ** 2) + 24 * Co * Se * So)
        assert abs(s3 - ref) < 1e-13 * scale
        co, se, so = r3 * Co, r3 * Se, r3 * So
        s3s = np.sum(4 * Ce * (Ce ** 2 + co ** 2 + se ** 2 + so ** 2)) + 8 / r3 * np.sum(co * se * so)
        assert abs(s3s - ref) < 1e-13 * scale
        # the four quadrant values are the offset grid's field
        jj = np.arange(N)
        xa = -math.pi + 2 * math.pi * (jj + 0.5) / N
        kk = np.arange(1, K + 1)
        uo = np.cos(np.outer(xa, kk)) @ x[:K] + np.sin(np.outer(xa, kk)) @ x[K:]
        A, B, A2, B2 = Ce + Co, Se + So, Ce - Co, Se - So
        q = N // 4
        assert np.allclose(uo[N // 2: N // 2 + q], A + B, atol=1e-12)        # xi in (0, pi/2)
        assert np.allclose(uo[N // 2 - q: N // 2][::-1], A - B, atol=1e-12)  # -xi
        assert np.allclose(uo[:q], A2 + B2, atol=1e-12)                      # xi - pi
        assert np.allclose(uo[N - q:][::-1], A2 - B2, atol=1e-12)            # pi - xi


def test_quarter_form_operand_layout_covers_every_coordinate_once():
    """K = 128 operands: lane group g (lanes 16g .. 16g + 15) holds the cos and
    sin coordinates of modes 32 g + 1 .. 32 g + 32; k-step r of an even-mode
    (odd-mode) contraction takes from group g the 8 modes 32 g + 2 (8 r + e) + 2
    (+ 1), e < 8.  Over the two k-steps of each of Ce, Co, Se, So every one of
    the 2K coordinates enters exactly once."""
    K = 128
    seen = np.zeros(2 * K, dtype=int)
    for block in (0, 1):                 # cos, sin
        for parity in (0, 1):            # even, odd
            for r in (0, 1):
                for g in range(4):
                    for e in range(8):
                        k = 32 * g + 2 * (8 * r + e) + (2 if parity == 0 else 1)
                        assert (k % 2 == 0) == (parity == 0)
                        seen[block * K + k - 1] += 1
    assert np.all(seen == 1)


@pytest.mark.parametrize("K", [64, 128])
def test_power_sums_from_the_orbits_and_the_grid_difference(K):
    """The SIR weights kernel at K = 128 forms S_p = sum_j u~^p, p = 1..4, from
    the four offset-grid syntheses (co, se, so carrying sqrt 3), with
    Q = Ce^2 + co^2 + se^2 + so^2, sg = co^2 + se^2 + so^2 and
    m = co^2 se^2 + co^2 so^2 + se^2 so^2 per representative:
        S1 = 4 sum Ce,  S2 = (4/3) sum (2 Ce^2 + Q),
        S4 = 4 sum (Q^2 - (8/9) sg^2 + (4/9) m) + (32/sqrt 3) sum Ce co se so,
    and carries S4 to the grid xi_j = -pi + 2 pi j/N by adding
    (N/4) (a^4 - 6 a^2 b^2 + b^4), a = x_K, b = x_2K (u~^4 reaches frequency N
    through the top mode alone; the two grids see it with opposite signs).
    S1..S3 need no correction (no frequency N)."""
    N = 4 * K
    rng = np.random.default_rng(K + 7)
    amp = math.sqrt(2.0 / math.pi)
    r3 = math.sqrt(3.0)
    for trial in range(12):
        x = rng.standard_normal(2 * K) / np.sqrt(1.0 + np.tile(np.arange(K), 2) ** (0.3 * (trial % 3)))
        if trial == 0:                       # the top mode alone: the difference at its largest
            x[:] = 0.0
            x[K - 1], x[2 * K - 1] = 0.6, 0.8
        x /= np.linalg.norm(x)
        u = oracle.grid(x, 1.0, N) / amp     # the grid xi_j
        Ce, Co, Se, So = _quarter_syntheses(x, K, N)
        co, se, so = r3 * Co, r3 * Se, r3 * So
        Q = Ce ** 2 + co ** 2 + se ** 2 + so ** 2
        sg = co ** 2 + se ** 2 + so ** 2
        m = co ** 2 * se ** 2 + co ** 2 * so ** 2 + se ** 2 * so ** 2
        S1 = 4 * np.sum(Ce)
        S2 = 4 / 3 * np.sum(2 * Ce ** 2 + Q)
        S3 = 4 * np.sum(Ce * Q) + 8 / r3 * np.sum(co * se * so)
        S4_off = 4 * np.sum(Q ** 2 - 8 / 9 * sg ** 2 + 4 / 9 * m) + 32 / r3 * np.sum(Ce * co * se * so)
        a, b = x[K - 1], x[2 * K - 1]
        S4 = S4_off + N / 4 * (a ** 4 - 6 * a ** 2 * b ** 2 + b ** 4)
        # the offset grid's own sums, directly
        jj = np.arange(N)
        xa = -math.pi + 2 * math.pi * (jj + 0.5) / N
        kk = np.arange(1, K + 1)
        uo = np.cos(np.outer(xa, kk)) @ x[:K] + np.sin(np.outer(xa, kk)) @ x[K:]
        scale = np.sum(u ** 4) + 1.0
        assert abs(S4_off - np.sum(uo ** 4)) < 1e-12 * scale
        assert abs(S1 - np.sum(u)) < 1e-12 * scale
        assert abs(S2 - np.sum(u ** 2)) < 1e-12 * scale
        assert abs(S3 - np.sum(u ** 3)) < 1e-12 * scale
        assert abs(S4 - np.sum(u ** 4)) < 1e-12 * scale
        if trial == 0:
            # u~ = 0.6 cos K xi + 0.8 sin K xi: the grids differ by (N/4) Re((a - ib)^4) != 0
            assert abs(np.sum(u ** 4) - np.sum(uo ** 4)) > 0.1 * N


@pytest.mark.parametrize("K", [64, 128])
def test_statistics_grid_orbits_cover_every_index_once(K):
    """On the grid xi_j = -pi + 2 pi j/N itself (the statistics and the extremes
    search at K >= 64), representative rho < K at xi = 2 pi rho/N gives u~ at
    xi (index 2K + rho), xi - pi (rho), -xi (2K - rho) and pi - xi (4K - rho), the
    last two for rho > 0 only; +-pi/2 (indices 3K, K) come from direct sums
    (cos k pi/2 and sin k pi/2 are 0 or +-1).  Every index is reached exactly
    once, with the field values of those combinations."""
    N = 4 * K
    rng = np.random.default_rng(K + 3)
    x = rng.standard_normal(2 * K)
    x /= np.linalg.norm(x)
    u = oracle.grid(x, 1.0, N) / math.sqrt(2.0 / math.pi)
    k = np.arange(1, K + 1)
    ev = k % 2 == 0
    seen = np.zeros(N, dtype=int)
    for rho in range(K):
        xi = 2 * math.pi * rho / N
        c, s = np.cos(k * xi), np.sin(k * xi)
        Ce, Co = c[ev] @ x[:K][ev], c[~ev] @ x[:K][~ev]
        Se, So = s[ev] @ x[K:][ev], s[~ev] @ x[K:][~ev]
        pe, me, ps, ms = Ce + Co, Ce - Co, Se + So, Se - So
        pairs = [(2 * K + rho, pe + ps), (rho, me + ms)]
        if rho:
            pairs += [(2 * K - rho, pe - ps), (4 * K - rho, me - ms)]
        for j, val in pairs:
            seen[j] += 1
            assert abs(u[j] - val) < 1e-12
    A = np.sum(x[3:K:4] - x[1:K:4])            # sum_k a_k cos(k pi/2): k = 0 mod 4 minus k = 2 mod 4
    B = np.sum(x[K:2 * K:4] - x[K + 2:2 * K:4])  # sum_k b_k sin(k pi/2): k = 1 mod 4 minus k = 3 mod 4
    for j, val in ((3 * K, A + B), (K, A - B)):
        seen[j] += 1
        assert abs(u[j] - val) < 1e-12
    assert np.all(seen == 1)
