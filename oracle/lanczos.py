"""Lanczos tridiagonalisation in P-bit fixed point (test infrastructure).

Section 1 of the paper motivates the Hankel product by the Lanczos
iteration: repeated products with one symmetric matrix reduce it to a
tridiagonal one (coefficients alpha_j on the diagonal, beta_j beside it),
whose eigenvalues QR iterations then find.  The paper gives no fixed-point
form; this is the one the library computes, every operation exactly
defined on integers (value X * 2**-P) so that the GPU result is unique:

  q_0 = 0, q_1 given (|entries| <= 1), beta_1 = 0; for j = 1, 2, ...
    w       = A q_j                                  (the Hankel matvec, RNE)
    alpha_j = rne(sum_i q_j,i w_i)                   (one rounding of the exact dot)
    r_i     = rne(w_i - alpha_j q_j,i - beta_j q_j-1,i)   (one rounding per entry)
    nu      = rne(sum_i r_i^2)                       (|r|^2)
    stop if nu < 2**-120 (beta_{j+1} = 0: an invariant subspace, or a
         breakdown below what the scalars resolve)
    rho     = rsqrt(nu), a fixed Newton iteration (below)
    beta_{j+1} = rne(nu rho)                         (= sqrt(nu))
    q_{j+1,i}  = rne(r_i rho), clamped to [-1, 1]

rne(.) rounds an exact value to the nearest multiple of 2**-P, ties to
even.  rsqrt: with b = the bit length of nu's integer minus P (so that
2**(b-1) <= nu < 2**b) and s = ceil(b / 2), mu = nu 4**-s lies in [1/4, 1)
(exact when s <= 0, one rounding otherwise).  Newton's iteration for
1/sqrt(mu), y <- y (3 - mu y^2) / 2, runs with a working precision p that
doubles: p = min(P, 64) first, from y = 3/2, for 9 steps; then p grows to
min(P, 2p - 8) (y shifted up exactly) with one step per level, and two
steps at p = P.  A step at precision p rounds at 2**-p: rne(y y),
rne(mu_p (y y)) with mu_p = mu rounded to p bits, 3 - that, and rne of
(y times that) / 2.  Finally rho = y 2**-s (exact when s <= 0, rounded
otherwise).
"""
from __future__ import annotations

from . import fixedpoint as fp
from . import hankel


def rne(S: int, k: int) -> int:
    """S / 2**k to the nearest integer, ties to even (k >= 0)."""
    return fp.round_half_even(S, k) if k > 0 else S


NEWTON_START_BITS = 64      # working precision of the first Newton steps
NEWTON_START_STEPS = 9      # steps from y = 3/2 at that precision
NEWTON_FINAL_STEPS = 2      # steps at the full precision P


def newton_schedule(P: int) -> list:
    """(precision, steps) of the Newton levels for P fractional bits."""
    p = min(P, NEWTON_START_BITS)
    out = [(p, NEWTON_START_STEPS)]
    while p < P:
        p = min(P, 2 * p - 8)
        out.append((p, NEWTON_FINAL_STEPS if p == P else 1))
    return out


def rsqrt(N: int, P: int) -> int:
    """Fixed-point 1/sqrt(nu) for nu = N 2**-P > 0, by the fixed iteration."""
    b = N.bit_length() - P
    s = -((-b) // 2)                              # ceil(b / 2)
    M = rne(N, 2 * s) if s > 0 else N << (-2 * s)  # mu = M 2**-P in [1/4, 1]
    y, prev = 0, 0
    for p, steps in newton_schedule(P):
        y = 3 << (p - 1) if prev == 0 else y << (p - prev)
        Mp = rne(M, P - p)                        # mu at p bits
        three = 3 << p
        for _ in range(steps):
            t1 = rne(y * y, p)
            t2 = rne(Mp * t1, p)
            y = rne(y * (three - t2), p + 1)
        prev = p
    return rne(y, s) if s > 0 else y << (-s)


def lanczos(H: list, q1: list, P: int, steps: int):
    """(alphas, betas, basis): alphas[j] = alpha_{j+1}, betas[j] = beta_{j+2}
    (the last is 0 at a stop), basis[j] = q_{j+1}; all integers (value *
    2**-P).  Stops early at a breakdown."""
    n = len(q1)
    fp.check_range(H, P)
    fp.check_range(q1, P)
    lim = 1 << P
    Q, Qp, B = list(q1), [0] * n, 0
    alphas, betas, basis = [], [], []
    for _ in range(steps):
        basis.append(list(Q))
        Wv = hankel.matvec_ints("hankel", H, Q, P)
        A = rne(sum(q * w for q, w in zip(Q, Wv)), P)
        R = [rne((w << P) - A * q - B * qp, P) for w, q, qp in zip(Wv, Q, Qp)]
        N = rne(sum(r * r for r in R), P)
        alphas.append(A)
        if N < (1 << P) >> 120 or N == 0:
            betas.append(0)
            break
        rho = rsqrt(N, P)
        B = rne(N * rho, P)
        betas.append(B)
        Qp, Q = Q, [max(-lim, min(lim, rne(r * rho, P))) for r in R]
    return alphas, betas, basis
