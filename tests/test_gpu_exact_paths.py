"""NTT path and Karatsuba path (Algorithm 1 of Section 4) on the GPU against
the oracle; three-way agreement with the split-FFT path at the paper's
precision."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import alg1, fixedpoint as fp, hankel, kronecker
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _oneshot(kind, h, x, n, P, algo):
    from paper_1402_5287_amd import hmv
    y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
    ws = hmv.workspace(hmv.oneshot_workspace_bytes(kind, n, P, algo))
    hmv.matvec(kind, hmv.to_device(h), hmv.to_device(x), y, n, P, algo=algo, ws=ws)
    rc, flags, _ = hmv.read_status(ws)
    return hmv.to_host(y), rc, flags


@pytest.mark.parametrize("algo", ["ntt", "karatsuba"])
@pytest.mark.parametrize("n,P", [(1, 1), (1, 100), (2, 5), (3, 63), (5, 64), (7, 65), (17, 200),
                                 (33, 1000), (64, 3322), (100, 129), (130, 4096)])
def test_ragged_sizes(algo, n, P):
    need_gpu()
    for kind in ("hankel", "toeplitz", "circulant"):
        hl = n if kind == "circulant" else 2 * n - 1
        h = si.uniform(hl, P, (70, n, P))
        x = si.uniform(n, P, (71, n, P))
        announce(algo, kind, n, P)
        y, rc, flags = _oneshot(kind, h, x, n, P, algo)
        assert rc == 0 and flags == 0
        assert np.array_equal(y, hankel.matvec_words(kind, h, x, P)), (algo, kind, n, P)


@pytest.mark.parametrize("algo", ["ntt", "karatsuba"])
def test_extremes_and_ties(algo):
    need_gpu()
    for P in (4, 64, 65, 3322):
        lim = 1 << P
        n = 6
        H = [lim if k % 2 else -lim for k in range(2 * n - 1)]
        X = [-lim, lim, lim, -lim, lim, lim]
        announce(algo, "extremes", P)
        y, rc, _ = _oneshot("hankel", fp.encode(H, P), fp.encode(X, P), n, P, algo)
        assert rc == 0
        assert np.array_equal(y, fp.encode(hankel.matvec_ints("hankel", H, X, P), P))
        for hv in (1, 3, 5, -1, -3, -5, -7):
            y, _, _ = _oneshot("hankel", fp.encode([hv], P), fp.encode([1 << (P - 1)], P), 1, P, algo)
            assert fp.decode(y) == [fp.round_half_even(hv << (P - 1), P)]


@pytest.mark.parametrize("algo", ["split_fft", "ntt", "karatsuba"])
def test_out_of_range_flag(algo):
    """Inputs must lie in [-1, 1] (|X| <= 2^P).  The values +-1 and +-(1 - 2^-P)
    pass; one step outside, in x or in h, sets the range flag and the call
    returns HMV_ERANGE.  P covers a top word used in part and in full."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n = 5
    for P in (62, 64, 100, 3322):
        lim = 1 << P
        h = si.uniform(2 * n - 1, P, (80, P))
        X = [lim, -lim, lim - 1, -(lim - 1), 0]
        announce(algo, "range ok", P)
        y, rc, flags = _oneshot("hankel", h, fp.encode(X, P), n, P, algo)
        assert rc == 0 and flags == 0
        assert np.array_equal(y, hankel.matvec_words("hankel", h, fp.encode(X, P), P))
        for bad in (lim + 1, -(lim + 1), 2 * lim, -2 * lim):
            announce(algo, "range x", P, bad > 0)
            _, rc, flags = _oneshot("hankel", h, fp.encode([0, 0, bad, 0, 0], P), n, P, algo)
            assert rc == hmv.ERANGE and (flags & 1), (P, bad)
        H = fp.decode(h)
        H[2 * n - 2] = -(lim + 1)
        announce(algo, "range h", P)
        # planning reads the flag of h at once: the call itself may return it
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        ws = hmv.workspace(hmv.oneshot_workspace_bytes("hankel", n, P, algo))
        call_rc = hmv.matvec("hankel", hmv.to_device(fp.encode(H, P)), hmv.to_device(fp.encode(X, P)),
                             y, n, P, algo=algo, ws=ws, check=False)
        rc, flags, _ = hmv.read_status(ws)
        assert hmv.ERANGE in (call_rc, rc) and (flags & 1)


def test_karatsuba_matches_algorithm1_sizes():
    """Sizes where Algorithm 1's halving is uneven (m != m1) at several levels."""
    need_gpu()
    for n in (33, 63, 65, 127, 129, 200, 257):
        P = 700
        h = si.uniform(2 * n - 1, P, (72, n))
        x = si.uniform(n, P, (73, n))
        announce("karatsuba", n)
        y, rc, _ = _oneshot("hankel", h, x, n, P, "karatsuba")
        H, X = fp.decode(h), fp.decode(x)
        want = [fp.round_half_even(s, P) for s in alg1.alg1(n, H, X)]
        assert fp.decode(y) == want


def test_auto_falls_back_to_ntt():
    """With the binary64 width forced above what the bound allows, AUTO plans
    the NTT path and the result is still exact."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 300, 3322
    h = si.uniform(2 * n - 1, P, (74,))
    x = si.uniform(n, P, (75,))
    hmv.force_width(20)
    try:
        plan = hmv.Plan("hankel", hmv.to_device(h), n, P, algo="auto")
        assert plan.info()["algo"] == hmv.NTT
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        plan.matvec(hmv.to_device(x), y)
        assert np.array_equal(hmv.to_host(y), hankel.matvec_words("hankel", h, x, P))
        plan.close()
    finally:
        hmv.force_width(0)


def test_three_way_hilbert_n1024_p33220():
    """n = 1024, P = 33220, Hilbert h: split-FFT, NTT and Karatsuba agree bit
    for bit, and with the exact GMP product."""
    need_gpu()
    n, P = 1024, 33220
    h, x = si.hilbert_case(n, P, seed=0)
    outs = {}
    for algo in ("split_fft", "ntt", "karatsuba"):
        announce("three-way", algo)
        y, rc, flags = _oneshot("hankel", h, x, n, P, algo)
        assert rc == 0 and flags == 0, algo
        outs[algo] = y
    assert np.array_equal(outs["split_fft"], outs["ntt"])
    assert np.array_equal(outs["split_fft"], outs["karatsuba"])
    if kronecker.available():
        assert np.array_equal(outs["ntt"], kronecker.hankel_matvec_words(h, x, P))
    rows = [0, 5, 1023]
    H, X = fp.decode(h), fp.decode(x)
    assert fp.decode(outs["karatsuba"][rows]) == hankel.matvec_rows("hankel", H, X, P, rows, processes=4)
