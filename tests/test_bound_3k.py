"""The error bound's stage charges for limb transforms of 3K points and for
the packed real column, checked by replaying the products in binary64 at
small sizes (CPU only).

The replay follows the kernels' formulas for the radix-3 split and its
inverse recombination (rounded sqrt(3)/2 and sqrt(3), tabulated roots of
order 3K), the real-input packing and unpacking of the K-point transform,
the two-real-bins column (x side: (U +- U*) products and a sum; h side:
(H +- H*) / 4 with the 1/(N_t N_z) scale), and the 1/3 scaling of the
resident spectrum; its complex transforms are radix-2 Stockham stages with
correctly rounded roots (one rounded sum and one rounded root product per
stage, Percival's operation model).  Every computed coefficient is compared
with the exact integer correlation of all-extreme digits; the largest
distance must stay below the bound the planner charges,
  |a|_2 |b|_2 ((1+e)^(3k) (1+e sqrt5)^(3k+1) (1+beta)^(3k) - 1),
  k = log2 N_t + log2 K + 2 (radix-3) + 1 (1/3) + 2 (packing) [+ 1 packed].
"""
import math

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

EPS = 2.0 ** -53


def _root_table(N):
    """exp(-2 pi i m / N), m < N, correctly rounded to binary64, and their
    largest error."""
    mpmath.mp.prec = 120
    out = np.empty(N, dtype=np.complex128)
    worst = 0.0
    for m in range(N):
        th = -2 * mpmath.pi * m / N
        c, s = mpmath.cos(th), mpmath.sin(th)
        out[m] = complex(float(c), float(s))
        worst = max(worst, float(mpmath.sqrt((out[m].real - c) ** 2 + (out[m].imag - s) ** 2)))
    return out, worst


def _fft(x, sign, roots_cache):
    """Unnormalised radix-2 Stockham transform along axis 0 (sign -1 forward)."""
    N = x.shape[0]
    if N == 1:
        return x.copy()
    if N not in roots_cache:
        roots_cache[N] = _root_table(N)
    w = roots_cache[N][0]
    if sign > 0:
        w = np.conj(w)
    a = x.copy()
    Ns = 1
    while Ns < N:
        half = N // 2
        b = np.empty_like(a)
        for j in range(half):
            k = j % Ns
            tw = w[(k * (N // (2 * Ns))) % N]
            u = a[j]
            v = a[j + half] * tw if Ns > 1 or k else a[j + half]
            base = (j - k) * 2 + k
            b[base] = u + v
            b[base + Ns] = u - v
        a = b
        Ns *= 2
    return a


def _real_fwd_K(u0, K, rc):
    """Real K-point transform of the columns of u0 (K x cols) as a K/2-point
    complex transform plus the packing step: bins 0..K/2."""
    z = u0[0::2] + 1j * u0[1::2]
    Z = _fft(z, -1, rc)
    if K not in rc:
        rc[K] = _root_table(K)
    wK = rc[K][0]
    out = np.empty((K // 2 + 1,) + u0.shape[1:], dtype=np.complex128)
    M = K // 2
    for k in range(M + 1):
        zk, zm = Z[k % M], Z[(M - k) % M]
        A = zk + np.conj(zm)
        B = zk - np.conj(zm)
        Q = wK[k % K] * B
        out[k] = 0.5 * (A.real + Q.imag) + 1j * (0.5 * (A.imag - Q.real))
    return out


def _real_inv_K(Y, K, rc):
    """Unnormalised inverse of _real_fwd_K (bins 0..K/2 -> K reals)."""
    M = K // 2
    wK = rc[K][0]
    Z = np.empty((M,) + Y.shape[1:], dtype=np.complex128)
    for k in range(M):
        yk, ym = Y[k], Y[M - k]
        E = yk + np.conj(ym)
        D = yk - np.conj(ym)
        Q = D * np.conj(wK[k])
        Z[k] = (E.real - Q.imag) + 1j * (E.imag + Q.real)
    z = _fft(Z, +1, rc)
    out = np.empty((K,) + Y.shape[1:], dtype=np.float64)
    out[0::2] = z.real
    out[1::2] = z.imag
    return out


S3H = float(mpmath.sqrt(3) / 2)
S3 = float(mpmath.sqrt(3))
THIRD = 1.0 / 3.0


def _fwd3(d, K, rc, r3):
    """Limb axis, forward: digits d (3K x rows, zero padded) -> (U0 bins 3m,
    U1 bins 3m+1)."""
    a, b, c = d[:K], d[K:2 * K], d[2 * K:]
    u0 = a + b + c
    re = a - 0.5 * (b + c)
    im = S3H * (c - b)
    u1 = (re + 1j * im) * r3[:, None]
    return _real_fwd_K(u0, K, rc), _fft(u1, -1, rc)


def _inv3(Y0, Y1, K, rc, r3):
    z0 = _real_inv_K(Y0, K, rc)
    z1 = _fft(Y1, +1, rc)
    v = z1 * np.conj(r3)[:, None]
    c0 = z0 + 2.0 * v.real
    c1 = (z0 - v.real) - S3 * v.imag
    c2 = (z0 - v.real) + S3 * v.imag
    return np.concatenate([c0, c1, c2], axis=0)


def _charged_bound(norm_h, norm_x, logNt, logK, pack, beta):
    k = logNt + logK + 2 + 1 + 2 + pack
    lg = 3 * k * math.log1p(EPS) + (3 * k + 1) * math.log1p(EPS * math.sqrt(5)) \
        + 3 * k * math.log1p(beta)
    return norm_h * norm_x * math.expm1(lg)


def _replay(n, K, w, pack, pattern):
    Nt = 1
    while Nt < 2 * n - 1:
        Nt *= 2
    Nz = 3 * K
    L = (Nz + 1) // 2                       # 2L - 1 <= 3K digits
    rng = np.random.default_rng(pattern)
    lim = 1 << (w - 1)
    if pattern == 0:
        Hd = np.full((2 * n - 1, L), -lim, dtype=np.int64)
        Xd = np.full((n, L), -lim, dtype=np.int64)
    else:
        Hd = rng.choice([-lim, lim - 1], size=(2 * n - 1, L)).astype(np.int64)
        Xd = rng.choice([-lim, lim - 1], size=(n, L)).astype(np.int64)
    # exact coefficients S[i][e] = sum_j sum_c H[i+j][c] X[j][e-c]
    S = np.zeros((n, 2 * L - 1), dtype=object)
    for i in range(n):
        for j in range(n):
            S[i] += np.convolve(Hd[i + j].astype(object), Xd[j].astype(object))
    rc = {}
    r3, b3 = _root_table(Nz)
    r3 = r3[:K]
    pad = lambda D: np.concatenate([D.T.astype(np.float64),
                                    np.zeros((Nz - D.shape[1], D.shape[0]))], axis=0)
    H0, H1 = _fwd3(pad(Hd), K, rc, r3)          # (K/2+1, 2n-1), (K, 2n-1)
    X0, X1 = _fwd3(pad(Xd), K, rc, r3)
    scale = THIRD * 2.0 ** -(int(math.log2(Nt)) + int(math.log2(K)))
    # index axis: columns are limb frequencies; rows 0..2n-2 of h, x reversed
    def index_fwd(cols, rows):
        buf = np.zeros((Nt, cols.shape[0]), dtype=np.complex128)
        buf[:rows] = cols.T
        return _fft(buf, -1, rc)
    Hc0, Hc1 = index_fwd(H0, 2 * n - 1), index_fwd(H1, 2 * n - 1)
    Xc0, Xc1 = index_fwd(X0[:, ::-1], n), index_fwd(X1[:, ::-1], n)
    Y1 = Xc1 * (Hc1 * scale)
    if pack:
        # column 0 carries bin 0 + i bin 3(K/2) (both real) on both sides
        xc = index_fwd((X0[0].real + 1j * X0[K // 2].real)[None, ::-1], n)[:, 0]
        hc = index_fwd((H0[0].real + 1j * H0[K // 2].real)[None, :], 2 * n - 1)[:, 0]
        part = lambda u: np.conj(u[(-np.arange(Nt)) % Nt])
        q = 0.25 * scale
        sa, sb = hc + part(hc), hc - part(hc)
        ha = sa * q
        hb = (sb.imag * q) + 1j * (-sb.real * q)
        ya = (xc + part(xc)) * ha + (xc - part(xc)) * hb
        Y0 = Xc0 * (Hc0 * scale)
        Y0[:, 0] = ya
        Y0[:, K // 2] = 0.0
    else:
        Y0 = Xc0 * (Hc0 * scale)
    y0 = _fft(Y0, +1, rc)[n - 1:2 * n - 1]     # rows n-1 .. 2n-2
    y1 = _fft(Y1, +1, rc)[n - 1:2 * n - 1]
    if pack:
        top = y0[:, 0].imag.copy()
        y0[:, 0] = y0[:, 0].real
        y0[:, K // 2] = top
    coef = _inv3(y0.T, y1.T, K, rc, r3)        # (3K, n)
    err = 0.0
    for i in range(n):
        for e in range(3 * K):
            exact = int(S[i][e]) if e < 2 * L - 1 else 0
            err = max(err, abs(coef[e, i] - exact))
    norm_h = math.sqrt(float(np.sum(Hd.astype(np.float64) ** 2)))
    norm_x = math.sqrt(float(np.sum(Xd.astype(np.float64) ** 2)))
    beta = max([b3] + [v[1] for v in rc.values()]) + 2.0 ** -60
    return err, _charged_bound(norm_h, norm_x, int(math.log2(Nt)), int(math.log2(K)), pack,
                               beta)


@pytest.mark.parametrize("n,K,pack", [(4, 16, 0), (4, 16, 1), (8, 32, 0), (8, 32, 1)])
def test_replayed_error_within_the_charged_bound(n, K, pack):
    # the largest width whose charged bound stays below 1/2 for these sizes
    for w in range(26, 8, -1):
        err, bound = _replay(n, K, w, pack, 0)
        if bound < 0.5:
            break
    assert bound < 0.5
    for pattern in (0, 1, 2):
        err, bound = _replay(n, K, w, pack, pattern)
        assert err < bound, (n, K, pack, w, pattern, err, bound)
        print(f"n={n} 3K={3 * K} pack={pack} w={w} pattern={pattern}: error {err:.3e}, "
              f"charged bound {bound:.3e}")
