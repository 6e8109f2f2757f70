"""Pins of the fixed-point Lanczos oracle (oracle/lanczos.py): closed forms
on matrices whose tridiagonal form is exact, the Newton reciprocal square
root against integer square roots, and the spectrum of the tridiagonal
matrix against the Hankel matrix's eigenvalues in high precision (CPU)."""
import random
from math import isqrt

import pytest

from oracle import lanczos


@pytest.mark.parametrize("P", [3, 64, 300])
def test_exchange_matrix(P):
    # h = e_{n-1}: A is the exchange matrix J; from q_1 = e_0 the iteration
    # finds J's 2-dimensional invariant subspace: alpha = 0, 0 and beta = 1, 0
    n = 4
    H = [0] * (2 * n - 1)
    H[n - 1] = 1 << P
    q1 = [1 << P, 0, 0, 0]
    a, b, basis = lanczos.lanczos(H, q1, P, 5)
    assert a == [0, 0] and b == [1 << P, 0]
    assert basis[1] == [0, 0, 0, 1 << P]


@pytest.mark.parametrize("P", [4, 65, 1000])
def test_rank_one_matrix(P):
    # h = 1/2 everywhere: A = (1/2) 1 1^T, n = 5, q_1 = e_0.  By hand:
    # w = 1/2 1, alpha_1 = 1/2, r = (0, 1/2, 1/2, 1/2, 1/2), |r| = 1,
    # q_2 = r, w_2 = 1, alpha_2 = 2, r_2 = 1 - 2 q_2 - e_0 = 0 (stop)
    n = 5
    half = 1 << (P - 1)
    H = [half] * (2 * n - 1)
    q1 = [1 << P] + [0] * (n - 1)
    a, b, basis = lanczos.lanczos(H, q1, P, 6)
    assert a == [half, 2 << P]
    assert b == [1 << P, 0]
    assert basis[1] == [0, half, half, half, half]


def test_rsqrt_against_integer_square_roots():
    rng = random.Random(5)
    for _ in range(300):
        P = rng.choice([2, 5, 30, 64, 200, 1000])
        k = rng.randrange(-110, 30)          # nu around 2^k
        N = max(1, rng.randrange(1, 1 << (P + 40)) >> max(0, 40 - k))
        if N < (1 << P) >> 120:
            continue
        rho = lanczos.rsqrt(N, P)
        # rho ~ 2^P / sqrt(N 2^-P) = sqrt(2^(3P) / N); floor with 8 guard bits
        g = 8
        ref = isqrt((1 << (3 * P + 2 * g)) // N)
        # the Newton result is within a few units of the last place of
        # 1/sqrt(mu) (mu = nu 4^-s), i.e. 2^-s units of rho's last place
        b = N.bit_length() - P
        s = -((-b) // 2)
        assert abs((rho << g) - ref) <= (6 << g) << max(0, -s), (P, N, rho, ref >> g)


def test_rsqrt_exact_powers_of_four():
    for P in (2, 10, 333):
        for k in range(-20, 10):
            if P + 2 * k < 0 or k > P:
                continue
            N = 1 << (P + 2 * k)             # nu = 4^k, 1/sqrt(nu) = 2^-k
            want = (1 << P) >> k if k > 0 else (1 << P) << (-k)
            assert lanczos.rsqrt(N, P) == want, (P, k)


def _mp_eigs(H, n, P, mp):
    A = mp.matrix(n, n)
    for i in range(n):
        for j in range(n):
            A[i, j] = mp.mpf(H[i + j]) / mp.mpf(2) ** P
    return sorted(mp.eigsy(A)[0])


def _tridiag_eigs(a, b, P, mp):
    m = len(a)
    T = mp.matrix(m, m)
    for i in range(m):
        T[i, i] = mp.mpf(a[i]) / mp.mpf(2) ** P
        if i + 1 < m:
            T[i, i + 1] = T[i + 1, i] = mp.mpf(b[i]) / mp.mpf(2) ** P
    return sorted(mp.eigsy(T)[0])


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tridiagonal_spectrum_equals_matrix_spectrum(seed):
    """n steps on an n x n Hankel matrix: the tridiagonal matrix has A's
    eigenvalues, to the precision the P-bit arithmetic carries."""
    mp = pytest.importorskip("mpmath").mp
    rng = random.Random(seed)
    n, P = 6, 240
    H = [rng.randrange(-(1 << P), 1 << P) for _ in range(2 * n - 1)]
    q = [rng.randrange(-(1 << P), 1 << P) for _ in range(n)]
    # a unit start vector (to rounding)
    nrm = isqrt(sum(v * v for v in q))
    q1 = [v * (1 << P) // nrm for v in q]
    a, b, basis = lanczos.lanczos(H, q1, P, n)
    assert len(a) == n
    mp.prec = P + 64
    want = _mp_eigs(H, n, P, mp)
    got = _tridiag_eigs(a, b, P, mp)
    for x, y in zip(want, got):
        assert abs(x - y) < mp.mpf(2) ** (-P + 40), (x, y)
    # and the basis is orthonormal to the same precision
    for i in range(n):
        for j in range(n):
            d = sum(u * v for u, v in zip(basis[i], basis[j]))
            target = (1 << (2 * P)) if i == j else 0
            assert abs(d - target) < 1 << (2 * P - P + 40)


def test_planted_mistakes_fail_the_spectrum_pin(monkeypatch):
    """A dropped beta term or a wrong sign in the three-term recurrence
    changes the tridiagonal spectrum."""
    mp = pytest.importorskip("mpmath").mp
    rng = random.Random(9)
    n, P = 5, 200
    H = [rng.randrange(-(1 << P), 1 << P) for _ in range(2 * n - 1)]
    q = [rng.randrange(-(1 << P), 1 << P) for _ in range(n)]
    nrm = isqrt(sum(v * v for v in q))
    q1 = [v * (1 << P) // nrm for v in q]
    mp.prec = P + 64
    want = _mp_eigs(H, n, P, mp)
    src = lanczos.lanczos

    def variant(bad):
        def run(H, q1, P, steps):
            n = len(q1)
            lim = 1 << P
            Q, Qp, B = list(q1), [0] * n, 0
            alphas, betas = [], []
            for _ in range(steps):
                Wv = lanczos.hankel.matvec_ints("hankel", H, Q, P)
                A = lanczos.rne(sum(x * w for x, w in zip(Q, Wv)), P)
                if bad == "no_beta":
                    R = [lanczos.rne((w << P) - A * x, P) for w, x in zip(Wv, Q)]
                else:
                    R = [lanczos.rne((w << P) - A * x + B * y, P) for w, x, y in zip(Wv, Q, Qp)]
                N = lanczos.rne(sum(r * r for r in R), P)
                alphas.append(A)
                if N == 0:
                    betas.append(0)
                    break
                rho = lanczos.rsqrt(N, P)
                B = lanczos.rne(N * rho, P)
                betas.append(B)
                Qp, Q = Q, [max(-lim, min(lim, lanczos.rne(r * rho, P))) for r in R]
            return alphas, betas, None
        return run

    for bad in ("no_beta", "beta_sign"):
        monkeypatch.setattr(lanczos, "lanczos", variant(bad))
        a, b, _ = lanczos.lanczos(H, q1, P, n)
        got = _tridiag_eigs(a, b, P, mp)
        assert max(abs(x - y) for x, y in zip(want, got)) > 1e-6, bad
    monkeypatch.setattr(lanczos, "lanczos", src)
    a, b, _ = lanczos.lanczos(H, q1, P, n)
    got = _tridiag_eigs(a, b, P, mp)
    assert max(abs(x - y) for x, y in zip(want, got)) < mp.mpf(2) ** (-P + 40)
