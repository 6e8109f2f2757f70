"""Pins for the CPU oracle: checks against what the paper's definitions and
mathematics fix, independent of the oracle's own code paths."""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import seeded_inputs as si
from oracle import alg1, decomposition, fixedpoint as fp, hankel, kronecker


def _rand_vals(rng, count, P, extremes=True):
    lim = 1 << P
    out = []
    for _ in range(count):
        r = rng.random()
        if extremes and r < 0.1:
            out.append(rng.choice([lim, -lim, 0, 1, -1, lim - 1, -lim + 1]))
        else:
            out.append(rng.randint(-lim, lim))
    return out


def _matrix(kind, a, n):
    """The full matrix from the paper's 1-based displays, eqs. (1)-(3)."""
    A = [[None] * n for _ in range(n)]
    for i in range(1, n + 1):
        for j in range(1, n + 1):
            if kind == "hankel":
                A[i - 1][j - 1] = a[i + j - 1 - 1]          # a_{i+j-1}
            elif kind == "toeplitz":
                A[i - 1][j - 1] = a[n - i + j - 1]          # a_{n-i+j}
            else:
                A[i - 1][j - 1] = a[((i - j) % n) + 1 - 1]  # a_{((i-j) mod n)+1}
    return A


@pytest.mark.parametrize("kind", ["hankel", "toeplitz", "circulant"])
def test_fraction_bruteforce(kind):
    """Exact rationals from the matrix displays, rounded by Python's own
    round-half-even on Fractions, equal the oracle for n <= 8."""
    rng = random.Random(1234 + len(kind))
    for trial in range(60):
        n = rng.randint(1, 8)
        P = rng.randint(1, 90)
        alen = n if kind == "circulant" else 2 * n - 1
        a = _rand_vals(rng, alen, P)
        x = _rand_vals(rng, n, P)
        af = [Fraction(v, 1 << P) for v in a]
        xf = [Fraction(v, 1 << P) for v in x]
        A = _matrix(kind, af, n)
        y = [sum(A[i][j] * xf[j] for j in range(n)) for i in range(n)]
        want = [round(v * (1 << P)) for v in y]      # ties to even
        assert hankel.matvec_ints(kind, a, x, P) == want, (trial, n, P)


def test_word_roundtrip_and_range():
    rng = random.Random(5)
    for P in (1, 63, 64, 65, 127, 128, 3322):
        vals = _rand_vals(rng, 20, P)
        w = fp.encode(vals, P)
        assert w.shape == (20, (P + 127) // 64)
        assert fp.decode(w) == vals
        assert si.words_to_ints(si.ints_to_words(vals, P)) == vals
    with pytest.raises(ValueError):
        fp.check_range([(1 << 10) + 1], 10)
    with pytest.raises(ValueError):
        fp.check_range([-(1 << 10) - 1], 10)
    fp.check_range([1 << 10, -(1 << 10)], 10)


def test_uniform_generator_range():
    for P in (5, 64, 200):
        vals = fp.decode(si.uniform(500, P, (7, P)))
        assert all(-(1 << P) <= v < (1 << P) for v in vals)
        assert min(vals) < -(1 << (P - 2)) and max(vals) > (1 << (P - 2))


def test_special_cases_bit_exact():
    rng = random.Random(9)
    for n, P in ((1, 7), (5, 64), (13, 200), (32, 3322)):
        h = _rand_vals(rng, 2 * n - 1, P)
        for k in (0, n - 1, n // 2):
            x = [(1 << P) if j == k else 0 for j in range(n)]
            assert hankel.matvec_ints("hankel", h, x, P) == h[k:k + n]
        assert hankel.matvec_ints("hankel", h, [0] * n, P) == [0] * n
        c = rng.randint(-(1 << P), 1 << P)
        x = _rand_vals(rng, n, P)
        S = c * sum(x)
        assert hankel.matvec_ints("hankel", [c] * (2 * n - 1), x, P) == \
            [fp.round_half_even(S, P)] * n
    for P in (1, 3, 64, 100):
        a, x = rng.randint(-(1 << P), 1 << P), rng.randint(-(1 << P), 1 << P)
        assert hankel.matvec_ints("hankel", [a], [x], P) == [round(Fraction(a * x, 1 << P))]


def test_rounding_ties():
    """Worked tie cases: the product lands exactly half-way between two
    representable values and must go to the even one."""
    for P in (4, 10, 64, 65, 3322):
        half = 1 << (P - 1)          # x = 0.5
        assert hankel.matvec_ints("hankel", [1], [half], P) == [0]      # 0.5 ulp -> 0
        assert hankel.matvec_ints("hankel", [3], [half], P) == [2]      # 1.5 ulp -> 2
        assert hankel.matvec_ints("hankel", [5], [half], P) == [2]      # 2.5 ulp -> 2
        assert hankel.matvec_ints("hankel", [-1], [half], P) == [0]
        assert hankel.matvec_ints("hankel", [-3], [half], P) == [-2]
        assert hankel.matvec_ints("hankel", [-5], [half], P) == [-2]
        assert hankel.matvec_ints("hankel", [-7], [half], P) == [-4]


def _harmonic(k):
    return sum(Fraction(1, i) for i in range(1, k + 1))


def test_hilbert_closed_form_ones():
    """h_k = 1/(k+1), x = 1: y_i = H_{i+n} - H_i (harmonic numbers), up to the
    input rounding of h (n * 2**-(P+1)) plus the output rounding."""
    for n, P in ((1, 20), (7, 40), (16, 64), (40, 200)):
        h = fp.decode(si.hilbert(2 * n - 1, P))
        y = hankel.matvec_ints("hankel", h, [1 << P] * n, P)
        tol = Fraction(n + 1, 1 << (P + 1))
        for i in range(n):
            exact = _harmonic(i + n) - _harmonic(i)
            assert abs(Fraction(y[i], 1 << P) - exact) <= tol


def _inv_hilbert(n):
    """Integer inverse of the n x n Hilbert matrix 1/(i+j+1), closed form."""
    C = math.comb
    return [[(-1) ** (i + j) * (i + j + 1) * C(n + i, n - j - 1) * C(n + j, n - i - 1)
             * C(i + j, i) ** 2 for j in range(n)] for i in range(n)]


def test_hilbert_inverse_columns():
    """x = 2**-s * (column k of the integer inverse Hilbert matrix) gives
    y = 2**-s e_k up to the rounding of h."""
    P = 160
    for n in (1, 2, 3, 4, 5):
        inv = _inv_hilbert(n)
        # the closed form really is the inverse
        for i in range(n):
            for j in range(n):
                s = sum(Fraction(1, i + t + 1) * inv[t][j] for t in range(n))
                assert s == (1 if i == j else 0)
        h = fp.decode(si.hilbert(2 * n - 1, P))
        for k in range(n):
            col = [inv[j][k] for j in range(n)]
            s = max(abs(v) for v in col).bit_length()
            x = [v << (P - s) for v in col]          # exact: col * 2**-s
            y = hankel.matvec_ints("hankel", h, x, P)
            tol = Fraction(sum(abs(v) for v in x), 1 << (2 * P + 1)) + Fraction(1, 1 << (P + 1))
            for i in range(n):
                want = Fraction(1, 1 << s) if i == k else Fraction(0)
                assert abs(Fraction(y[i], 1 << P) - want) <= tol


def test_symmetric_form_invariant():
    """A_H is symmetric, so z . (A x) = x . (A z) exactly on the integer sums."""
    rng = random.Random(11)
    for n, P in ((3, 30), (17, 100), (50, 700)):
        h = _rand_vals(rng, 2 * n - 1, P)
        x = _rand_vals(rng, n, P)
        z = _rand_vals(rng, n, P)
        Sx = hankel.hankel_sums(h, x)
        Sz = hankel.hankel_sums(h, z)
        assert sum(a * b for a, b in zip(z, Sx)) == sum(a * b for a, b in zip(x, Sz))


def test_toeplitz_hankel_circulant_identities():
    rng = random.Random(12)
    for n, P in ((1, 9), (2, 9), (9, 77), (31, 300)):
        h = _rand_vals(rng, 2 * n - 1, P)
        x = _rand_vals(rng, n, P)
        yh = hankel.matvec_ints("hankel", h, x, P)
        yt = hankel.matvec_ints("toeplitz", h, x, P)
        assert yt == yh[::-1]                                      # rows reversed
        assert yh == hankel.matvec_ints("toeplitz", h[::-1], x[::-1], P)
        c = _rand_vals(rng, n, P)
        cext = [c[(-d) % n] for d in range(-(n - 1), n)]          # cext[n-1+d] = c[-d mod n]
        assert hankel.matvec_ints("circulant", c, x, P) == hankel.matvec_ints("toeplitz", cext, x, P)
        e0 = [1 << P] + [0] * (n - 1)
        assert hankel.matvec_ints("circulant", c, e0, P) == c


def test_circulant_diagonalisation():
    """y = IDFT(DFT(c) * DFT(x)) in high-precision complex arithmetic (mpmath)."""
    mpmath = pytest.importorskip("mpmath")
    rng = random.Random(13)
    for n, P in ((1, 40), (3, 60), (8, 100), (16, 128)):
        c = _rand_vals(rng, n, P, extremes=False)
        x = _rand_vals(rng, n, P, extremes=False)
        y = hankel.matvec_ints("circulant", c, x, P)
        with mpmath.workprec(P + 96):
            cf = [mpmath.mpf(v) / 2**P for v in c]
            xf = [mpmath.mpf(v) / 2**P for v in x]
            w = [mpmath.expj(-2 * mpmath.pi * k / n) for k in range(n)]
            C = [mpmath.fsum(cf[t] * w[(k * t) % n] for t in range(n)) for k in range(n)]
            X = [mpmath.fsum(xf[t] * w[(k * t) % n] for t in range(n)) for k in range(n)]
            Y = [C[k] * X[k] for k in range(n)]
            yy = [mpmath.fsum(Y[k] * mpmath.conj(w[(k * t) % n]) for k in range(n)) / n
                  for t in range(n)]
            for i in range(n):
                assert abs(yy[i].imag) < mpmath.mpf(2) ** (-P - 20)
                assert abs(mpmath.mpf(y[i]) / 2**P - yy[i].real) <= mpmath.mpf(2) ** (-P - 1) * 1.0001


def test_alg1_equals_schoolbook():
    rng = random.Random(14)
    for n in range(1, 129):
        a = [rng.randint(-10**6, 10**6) for _ in range(2 * n - 1)]
        x = [rng.randint(-10**6, 10**6) for _ in range(n)]
        want = hankel.hankel_sums(a, x)
        assert alg1.alg1(n, a, x) == want, n
        if n % 7 == 0:
            assert alg1.alg1(n, a, x, n0=8) == want, n


class _Counted(int):
    count = 0

    def __mul__(self, other):
        _Counted.count += 1
        return _Counted(int(self) * int(other))

    __rmul__ = __mul__

    def __add__(self, o):
        return _Counted(int(self) + int(o))

    __radd__ = __add__

    def __sub__(self, o):
        return _Counted(int(self) - int(o))

    def __rsub__(self, o):
        return _Counted(int(o) - int(self))


def test_alg1_multiplication_count():
    """The count recurrence equals the multiplications the recursion really
    performs, and grows like n**log2(3)."""
    rng = random.Random(15)
    for n in list(range(1, 40)) + [64, 100, 128]:
        a = [_Counted(rng.randint(1, 9)) for _ in range(2 * n - 1)]
        x = [_Counted(rng.randint(1, 9)) for _ in range(n)]
        _Counted.count = 0
        alg1.alg1(n, a, x)
        assert _Counted.count == alg1.mult_count(n), n
    M = alg1.mult_count
    assert [M(k) for k in (4, 16, 18, 19, 32, 1024, 4096)] == \
        [20, 260, 332, 348, 844, 232100, 2109380]
    assert min(k for k in range(3, 5000) if M(k) < k * k) == 19
    assert all(M(k) < k * k for k in range(19, 4097))
    assert M(1024, n0=32) == 215705
    r = M(2**14) / M(2**13)
    assert abs(r - 3.0) < 0.05


def test_decomposition_exact_analogue():
    """The exact limb (decomposition) form: evaluating the bivariate
    index-by-limb correlation at z = 2**w gives the Hankel sums."""
    rng = random.Random(16)
    for n, P, w in ((1, 20, 4), (4, 64, 11), (7, 150, 16), (5, 33, 7)):
        L = -(-(P + 2) // w)
        h = _rand_vals(rng, 2 * n - 1, P)
        x = _rand_vals(rng, n, P)
        for v in h + x:
            d = decomposition.balanced_digits(v, w, L)
            assert all(-(1 << (w - 1)) <= t < (1 << (w - 1)) for t in d)
            assert decomposition.evaluate(d, w) == v
        coeffs = decomposition.hankel_limb_coeffs(h, x, w, L)
        S = hankel.hankel_sums(h, x)
        assert [decomposition.evaluate(c, w) for c in coeffs] == S
        bound = n * L * (1 << (2 * (w - 1)))
        assert all(abs(c) <= bound for row in coeffs for c in row)


@pytest.mark.skipif(not kronecker.available(), reason="libgmp not present")
def test_kronecker_equals_schoolbook():
    for n, P, seed in ((1, 5, 0), (2, 64, 1), (3, 63, 2), (64, 3322, 3), (257, 200, 4),
                       (300, 1024, 5)):
        h = si.uniform(2 * n - 1, P, (77, seed))
        x = si.uniform(n, P, (78, seed))
        if seed == 2:       # extreme values
            h[:] = si.ints_to_words([1 << P] * (2 * n - 1), P)
            x[:] = si.ints_to_words([-(1 << P)] * n, P)
        want = hankel.hankel_sums(fp.decode(h), fp.decode(x))
        assert kronecker.hankel_sums(h, x, P) == want


@pytest.mark.skipif(not kronecker.available(), reason="libgmp not present")
def test_kronecker_equals_schoolbook_n1024():
    """The Kronecker cross-check against the plain sums at n = 1024 (every
    row), the size it must reach before it is trusted at n = 4096."""
    n, P = 1024, 1024
    h = si.uniform(2 * n - 1, P, (79, 0))
    x = si.uniform(n, P, (79, 1))
    assert kronecker.hankel_sums(h, x, P) == hankel.hankel_sums(fp.decode(h), fp.decode(x))


@pytest.mark.skipif(not kronecker.available(), reason="libgmp not present")
def test_kronecker_rows_at_headline_size():
    """n = 4096, P = 33220: the Kronecker product equals the plain row sums
    on sampled rows (first, an interior one, last), computed over a pool."""
    n, P = 4096, 33220
    h = si.uniform(2 * n - 1, P, (80, 0))
    x = si.uniform(n, P, (80, 1))
    rows = [0, 1777, n - 1]
    sums = kronecker.hankel_sums(h, x, P)
    got = [fp.round_half_even(sums[i], P) for i in rows]
    assert got == hankel.matvec_rows("hankel", fp.decode(h), fp.decode(x), P, rows, processes=3)


def test_kronecker_range_checks_every_entry():
    n, P = 6, 64
    h = si.uniform(2 * n - 1, P, (81, 0))
    x = si.uniform(n, P, (81, 1))
    for arr, k in ((h, 2 * n - 2), (x, n - 1), (x, 0)):
        bad = arr.copy()
        bad[k:k + 1] = si.ints_to_words([(1 << P) + 1], P)
        args = (bad, x) if arr is h else (h, bad)
        with pytest.raises(ValueError):
            kronecker.hankel_sums(args[0], args[1], P)


@pytest.mark.parametrize("kind", ["hankel", "toeplitz", "circulant"])
@pytest.mark.parametrize("processes", [1, 4])
def test_row_sampled_oracle_equals_full_oracle(kind, processes):
    """matvec_rows (the row-sampled oracle behind every large-n check) equals
    matvec_ints row by row, for all three matrix kinds; at n <= 8 both also
    equal exact rationals from the matrix displays."""
    rng = random.Random(31 + processes + len(kind))
    for n, P in ((1, 9), (2, 64), (7, 65), (33, 200), (300, 130)):
        alen = n if kind == "circulant" else 2 * n - 1
        a = _rand_vals(rng, alen, P)
        x = _rand_vals(rng, n, P)
        full = hankel.matvec_ints(kind, a, x, P)
        rows = list(range(n)) if n <= 33 else sorted(rng.sample(range(n), 40) + [0, n - 1])
        assert hankel.matvec_rows(kind, a, x, P, rows, processes=processes) == \
            [full[i] for i in rows], (kind, n)
        if n <= 8:
            A = _matrix(kind, [Fraction(v, 1 << P) for v in a], n)
            xf = [Fraction(v, 1 << P) for v in x]
            assert full == [round(sum(A[i][j] * xf[j] for j in range(n)) * (1 << P))
                            for i in range(n)]


# ---------------------------------------------------------------------------
# planted mistakes: each pin above must reject a plausible wrong oracle
# ---------------------------------------------------------------------------

def test_pins_reject_planted_mistakes(monkeypatch):
    rng = random.Random(17)
    n, P = 5, 40
    a = _rand_vals(rng, 2 * n - 1, P, extremes=False)
    x = _rand_vals(rng, n, P, extremes=False)
    af = [Fraction(v, 1 << P) for v in a]
    xf = [Fraction(v, 1 << P) for v in x]
    A = _matrix("hankel", af, n)
    want = [round(sum(A[i][j] * xf[j] for j in range(n)) * (1 << P)) for i in range(n)]

    # (1) off-by-one anti-diagonal index
    monkeypatch.setitem(hankel._SUMS, "hankel",
                        lambda H, X: [sum(H[min(i + j + 1, len(H) - 1)] * X[j] for j in range(len(X)))
                                      for i in range(len(X))])
    assert hankel.matvec_ints("hankel", a, x, P) != want
    monkeypatch.undo()
    # (2) Toeplitz with the wrong orientation (columns reversed instead of rows)
    monkeypatch.setitem(hankel._SUMS, "toeplitz",
                        lambda H, X: [sum(H[i + (len(X) - 1 - j)] * X[j] for j in range(len(X)))
                                      for i in range(len(X))])
    At = _matrix("toeplitz", af, n)
    want_t = [round(sum(At[i][j] * xf[j] for j in range(n)) * (1 << P)) for i in range(n)]
    assert hankel.matvec_ints("toeplitz", a, x, P) != want_t
    monkeypatch.undo()
    # (3) rounding ties away from zero instead of to even
    monkeypatch.setattr(fp, "round_half_even",
                        lambda S, P: (S + (1 << (P - 1))) >> P if S >= 0 else -((-S + (1 << (P - 1))) >> P))
    assert hankel.matvec_ints("hankel", [5], [1 << 9], 10) != [2]
    monkeypatch.undo()
    # (4) Algorithm 1 with a sign error in the combine of its second row
    orig = alg1._half_products

    def bad(aa, xx, n0):
        y = orig(aa, xx, n0)
        if len(xx) > n0 and len(xx) >= 4:
            y[1] = -y[1]
        return y
    monkeypatch.setattr(alg1, "_half_products", bad)
    assert alg1.alg1(9, list(range(1, 18)), list(range(1, 10))) != \
        hankel.hankel_sums(list(range(1, 18)), list(range(1, 10)))
    monkeypatch.undo()
    # (5) the row-sampled oracle with a wrong circulant index ((i + j) mod n)
    orig_row = hankel._row_value

    def bad_row(kind, H, X, i, P):
        if kind == "circulant":
            nn = len(X)
            return fp.round_half_even(sum(H[(i + j) % nn] * X[j] for j in range(nn)), P)
        return orig_row(kind, H, X, i, P)
    monkeypatch.setattr(hankel, "_row_value", bad_row)
    c = [5, -3, 11, 2]
    xx = [1, 4, -2, 7]
    assert hankel.matvec_rows("circulant", c, xx, 4, range(4)) != \
        hankel.matvec_ints("circulant", c, xx, 4)
