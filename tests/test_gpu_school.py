"""GPU schoolbook path (the plain sum of Section 2) against the oracle,
bit-exact, through the C ABI; every test runs both forms (binary64 limb sums
on the vector units, int8 limb products on the matrix cores)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import fixedpoint as fp, hankel
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=[0, 1], ids=["vector", "mfma"])
def school_form(request):
    from paper_1402_5287_amd import hmv
    try:
        hmv.lib()
    except ImportError:
        yield request.param
        return
    hmv.force_school(request.param)
    try:
        yield request.param
    finally:
        hmv.force_school(-1)


def _run(kind, h, x, n, P, algo="schoolbook"):
    from paper_1402_5287_amd import hmv
    hd, xd = hmv.to_device(h), hmv.to_device(x)
    y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
    ws = hmv.workspace(hmv.oneshot_workspace_bytes(kind, n, P, algo))
    hmv.matvec(kind, hd, xd, y, n, P, algo=algo, ws=ws)
    rc, flags, _ = hmv.read_status(ws)
    return hmv.to_host(y), rc, flags


@pytest.mark.parametrize("kind", ["hankel", "toeplitz", "circulant"])
def test_plain_n64_p3322(kind):
    need_gpu()
    n, P = 64, 3322
    h, x = si.plain_case(n, P, seed=0)
    if kind == "circulant":
        h = h[:n].copy()
    announce("school", kind, n, P)
    y, rc, flags = _run(kind, h, x, n, P)
    assert rc == 0 and flags == 0
    want = hankel.matvec_words(kind, h, x, P)
    assert np.array_equal(y, want)


@pytest.mark.parametrize("n,P", [(1, 1), (1, 64), (2, 5), (3, 63), (5, 64), (7, 65), (17, 200),
                                 (33, 1000), (100, 129), (130, 4096)])
def test_ragged_sizes(n, P):
    need_gpu()
    for kind in ("hankel", "toeplitz", "circulant"):
        hl = n if kind == "circulant" else 2 * n - 1
        h = si.uniform(hl, P, (50, n, P))
        x = si.uniform(n, P, (51, n, P))
        announce("school ragged", kind, n, P)
        y, rc, flags = _run(kind, h, x, n, P)
        assert rc == 0 and flags == 0
        assert np.array_equal(y, hankel.matvec_words(kind, h, x, P)), (kind, n, P)


def test_extremes_and_ties():
    need_gpu()
    for P in (4, 64, 65, 3322):
        lim = 1 << P
        n = 6
        # all +-1 entries: largest magnitudes, exact integer outputs
        H = [lim if k % 2 else -lim for k in range(2 * n - 1)]
        X = [-lim, lim, lim, -lim, lim, lim]
        announce("school extremes", P)
        y, rc, _ = _run("hankel", fp.encode(H, P), fp.encode(X, P), n, P)
        assert rc == 0
        assert np.array_equal(y, fp.encode(hankel.matvec_ints("hankel", H, X, P), P))
        # ties: h = k ulp, x = 0.5
        H = [k - 5 for k in range(2 * 1 - 1 + 10)][:1]
        for hv in (1, 3, 5, -1, -3, -5, -7):
            y, rc, _ = _run("hankel", fp.encode([hv], P), fp.encode([1 << (P - 1)], P), 1, P)
            assert fp.decode(y) == [fp.round_half_even(hv << (P - 1), P)]


def test_basis_vectors_bit_exact():
    need_gpu()
    n, P = 40, 700
    h = si.uniform(2 * n - 1, P, (52,))
    H = fp.decode(h)
    for k in (0, 13, n - 1):
        announce("school basis", k)
        y, rc, _ = _run("hankel", h, si.unit(n, P, k), n, P)
        assert fp.decode(y) == H[k:k + n]


def test_largest_n():
    """n = HMV_MAX_N (16384), the schoolbook's limit, at a one-word precision;
    sampled rows against the oracle."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = hmv.MAX_N, 64
    h = si.uniform(2 * n - 1, P, (76,))
    x = si.uniform(n, P, (77,))
    announce("school largest n", n, P)
    y, rc, flags = _run("hankel", h, x, n, P)
    assert rc == 0 and flags == 0
    rows = [0, 1, n // 2, n - 1]
    H, X = fp.decode(h), fp.decode(x)
    assert fp.decode(y[rows]) == hankel.matvec_rows("hankel", H, X, P, rows, processes=4)


def test_out_of_range_flag():
    need_gpu()
    n, P = 4, 100
    h = si.uniform(2 * n - 1, P, (53,))
    x = fp.encode([1, 2, (1 << P) + 1, 0], P)
    announce("school range")
    _, rc, flags = _run("hankel", h, x, n, P)
    assert rc == -2 and (flags & 1)


@pytest.mark.parametrize("n,P", [(3, 40960), (70, 33220), (300, 8), (257, 2000)])
def test_paper_precisions(n, P, school_form):
    """Large precisions (the MFMA form's LDS row at P = 40960 is its largest)
    and index lengths across a 64-row stage boundary."""
    need_gpu()
    for kind in ("hankel", "circulant"):
        hl = n if kind == "circulant" else 2 * n - 1
        h = si.uniform(hl, P, (54, n, P))
        x = si.uniform(n, P, (55, n, P))
        announce("school precisions", school_form, kind, n, P)
        y, rc, flags = _run(kind, h, x, n, P)
        assert rc == 0 and flags == 0
        assert np.array_equal(y, hankel.matvec_words(kind, h, x, P)), (kind, n, P)


def test_forms_agree_at_n1024_p33220(school_form):
    """Both forms give identical words on a paper-sized product (the oracle
    is checked on sampled rows)."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    if school_form == 0:
        pytest.skip("compared once, from the MFMA parametrisation")
    n, P = 1024, 33220
    h = si.uniform(2 * n - 1, P, (56,))
    x = si.uniform(n, P, (57,))
    announce("school forms agree", n, P)
    y1, rc1, f1 = _run("toeplitz", h, x, n, P)
    hmv.force_school(0)
    y0, rc0, f0 = _run("toeplitz", h, x, n, P)
    assert rc0 == rc1 == 0 and f0 == f1 == 0
    assert np.array_equal(y0, y1)
    rows = [0, 511, n - 1]
    assert fp.decode(y1[rows]) == hankel.matvec_rows("toeplitz", fp.decode(h), fp.decode(x), P,
                                                     rows, processes=3)
