"""The identities behind the split-FFT spectrum layouts, checked in numpy
against direct transforms (no GPU, no oracle): the radix-3 split of a real
transform of N = 3K points into a real and a complex K-point transform, its
inverse recombination, and the product of the packed column that carries the
two real limb bins.  The GPU kernels compute exactly these expressions."""
import numpy as np


def _split3(x, K):
    """Bins 3m (m <= K/2) and 3m+1 (m < K) of the real N = 3K point DFT of x."""
    N = 3 * K
    a, b, c = x[:K], x[K:2 * K], x[2 * K:]
    s = np.arange(K)
    u0 = a + b + c
    u1 = ((a - 0.5 * (b + c)) + 1j * (np.sqrt(3) / 2) * (c - b)) * np.exp(-2j * np.pi * s / N)
    return np.fft.fft(u0)[:K // 2 + 1], np.fft.fft(u1)


def _join3(Z0, Z1, K):
    """N x from bins 3m (m <= K/2) and 3m+1 of a real sequence's DFT."""
    N = 3 * K
    full0 = np.concatenate([Z0, np.conj(Z0[1:K // 2][::-1])])
    z0 = np.fft.ifft(full0).real * K
    z1 = np.fft.ifft(Z1) * K
    v = z1 * np.exp(2j * np.pi * np.arange(K) / N)
    return np.concatenate([z0 + 2 * v.real, z0 - v.real - np.sqrt(3) * v.imag,
                           z0 - v.real + np.sqrt(3) * v.imag])


def test_radix3_split_matches_direct_transform():
    rng = np.random.default_rng(3)
    for K in (64, 128, 2048):
        N = 3 * K
        x = np.zeros(N)
        L = (N + 1) // 2 - 5
        x[:L] = rng.integers(-1024, 1024, L)
        Z0, Z1 = _split3(x, K)
        F = np.fft.fft(x)
        scale = np.abs(F).max()
        assert np.abs(Z0 - F[0::3][:K // 2 + 1]).max() < 1e-12 * scale
        assert np.abs(Z1 - F[1::3]).max() < 1e-12 * scale
        # bins 3m+2 are the conjugates of bins 3(K-1-m)+1 (real input)
        assert np.abs(F[2::3] - np.conj(F[1::3][::-1])).max() < 1e-12 * scale


def test_radix3_inverse_gives_linear_convolution():
    rng = np.random.default_rng(4)
    K = 256
    N = 3 * K
    L = (N + 1) // 2                     # 2L - 1 <= N: the linear product fits
    x = np.zeros(N)
    h = np.zeros(N)
    x[:L] = rng.integers(-1024, 1024, L)
    h[:L] = rng.integers(-1024, 1024, L)
    X0, X1 = _split3(x, K)
    H0, H1 = _split3(h, K)
    y = _join3(X0 * H0, X1 * H1, K) / N
    assert np.array_equal(np.rint(y), np.convolve(x, h)[:N])
    assert np.abs(y - np.rint(y)).max() < 1e-6


def test_packed_real_column_product():
    """Column 0 carries c = a + i b (a, b: the real columns of limb bins 0 and
    N_z/2).  With U its index transform, U*[k] = conj U[N - k], and Ha, Hb the
    index transforms of h's two real columns, (U + U*) Ha/2 + (U - U*) Hb/2
    equals A Ha + i B Hb, whose inverse is the pair of real products."""
    rng = np.random.default_rng(5)
    Nt = 64
    a, b, ha, hb = (rng.standard_normal(Nt) for _ in range(4))
    U = np.fft.fft(a + 1j * b)
    Ustar = np.conj(U[(-np.arange(Nt)) % Nt])
    Hc = np.fft.fft(ha + 1j * hb)
    Hcstar = np.conj(Hc[(-np.arange(Nt)) % Nt])
    Ha2 = (Hc + Hcstar) / 4                 # Ha / 2
    Hb2 = -1j * (Hc - Hcstar) / 4           # Hb / 2
    V = (U + Ustar) * Ha2 + (U - Ustar) * Hb2
    want = np.fft.fft(a) * np.fft.fft(ha) + 1j * np.fft.fft(b) * np.fft.fft(hb)
    assert np.abs(V - want).max() < 1e-12 * np.abs(want).max()
    y = np.fft.ifft(V)
    ya = np.real(np.fft.ifft(np.fft.fft(a) * np.fft.fft(ha)))
    yb = np.real(np.fft.ifft(np.fft.fft(b) * np.fft.fft(hb)))
    assert np.abs(y.real - ya).max() < 1e-12 and np.abs(y.imag - yb).max() < 1e-12
    # partner bins inside the even / odd halves of the index transform
    Nh = Nt // 2
    E, O = U[0::2], U[1::2]
    k = np.arange(Nh)
    assert np.allclose(Ustar[0::2], np.conj(E[(Nh - k) % Nh]))
    assert np.allclose(Ustar[1::2], np.conj(O[Nh - 1 - k]))
