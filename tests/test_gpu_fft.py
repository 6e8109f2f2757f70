"""Split-FFT path (Section 3 decomposition, exact form) on the GPU against
the oracle: bit-exact at small sizes, sampled rows plus the GMP Kronecker
full-vector cross-check at the paper-shaped sizes."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import fixedpoint as fp, hankel, kronecker
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _oneshot(kind, h, x, n, P, algo="split_fft"):
    from paper_1402_5287_amd import hmv
    y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
    ws = hmv.workspace(hmv.oneshot_workspace_bytes(kind, n, P, algo))
    hmv.matvec(kind, hmv.to_device(h), hmv.to_device(x), y, n, P, algo=algo, ws=ws)
    rc, flags, err = hmv.read_status(ws)
    return hmv.to_host(y), rc, flags, err


@pytest.mark.parametrize("kind", ["hankel", "toeplitz", "circulant"])
def test_plain_n64_p3322(kind):
    need_gpu()
    n, P = 64, 3322
    h, x = si.plain_case(n, P, seed=0)
    if kind == "circulant":
        h = h[:n].copy()
    announce("fft oneshot", kind, n, P)
    y, rc, flags, err = _oneshot(kind, h, x, n, P)
    assert rc == 0 and flags == 0
    assert err < 0.25
    assert np.array_equal(y, hankel.matvec_words(kind, h, x, P))


@pytest.mark.parametrize("n,P", [(1, 1), (1, 100), (2, 5), (3, 63), (5, 64), (7, 65), (17, 200),
                                 (33, 1000), (100, 129), (130, 4096), (257, 3322)])
def test_ragged_sizes(n, P):
    need_gpu()
    for kind in ("hankel", "toeplitz", "circulant"):
        hl = n if kind == "circulant" else 2 * n - 1
        h = si.uniform(hl, P, (60, n, P))
        x = si.uniform(n, P, (61, n, P))
        announce("fft ragged", kind, n, P)
        y, rc, flags, _ = _oneshot(kind, h, x, n, P)
        assert rc == 0 and flags == 0
        assert np.array_equal(y, hankel.matvec_words(kind, h, x, P)), (kind, n, P)


def test_extremes_basis_ties():
    need_gpu()
    for P in (4, 64, 65, 3322):
        lim = 1 << P
        n = 6
        H = [lim if k % 2 else -lim for k in range(2 * n - 1)]
        X = [-lim, lim, lim, -lim, lim, lim]
        announce("fft extremes", P)
        y, rc, _, _ = _oneshot("hankel", fp.encode(H, P), fp.encode(X, P), n, P)
        assert rc == 0
        assert np.array_equal(y, fp.encode(hankel.matvec_ints("hankel", H, X, P), P))
        for hv in (1, 3, 5, -1, -3, -5, -7):
            y, rc, _, _ = _oneshot("hankel", fp.encode([hv], P), fp.encode([1 << (P - 1)], P), 1, P)
            assert fp.decode(y) == [fp.round_half_even(hv << (P - 1), P)]
    n, P = 300, 2000
    h = si.uniform(2 * n - 1, P, (62,))
    H = fp.decode(h)
    for k in (0, 77, n - 1):
        y, rc, _, _ = _oneshot("hankel", h, si.unit(n, P, k), n, P)
        assert fp.decode(y) == H[k:k + n]


def test_planned_reuse_and_info():
    """One plan, several vectors: each result equals the oracle."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 200, 3322
    h = si.uniform(2 * n - 1, P, (63,))
    plan = hmv.Plan("hankel", hmv.to_device(h), n, P, algo="split_fft")
    info = plan.info()
    assert info["algo"] == 1 and info["bound"] < 0.5 and 8 <= info["w"] <= 20
    H = fp.decode(h)
    for k in range(3):
        x = si.uniform(n, P, (64, k))
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        announce("fft planned", k)
        plan.matvec(hmv.to_device(x), y)
        rc, flags, err = hmv.read_status(plan.ws)
        assert rc == 0 and err <= info["bound"]
        assert np.array_equal(hmv.to_host(y), fp.encode(hankel.matvec_ints("hankel", H, fp.decode(x), P), P))
    plan.close()


def test_forced_width_bound_refusal():
    """A limb width the proven bound rejects is refused (EBOUND)."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 1024, 33220
    h = si.uniform(2 * n - 1, P, (65,))
    hmv.force_width(20)
    try:
        with pytest.raises(hmv.HmvError) as ei:
            hmv.Plan("hankel", hmv.to_device(h), n, P, algo="split_fft")
        assert ei.value.code == hmv.EBOUND
    finally:
        hmv.force_width(0)


def test_cross_path_equals_schoolbook():
    need_gpu()
    n, P = 256, 4096
    h = si.uniform(2 * n - 1, P, (66,))
    x = si.uniform(n, P, (67,))
    announce("fft vs school", n, P)
    y1, *_ = _oneshot("hankel", h, x, n, P, "split_fft")
    y2, *_ = _oneshot("hankel", h, x, n, P, "schoolbook")
    assert np.array_equal(y1, y2)


def _sampled_rows_check(h, x, y, P, rows):
    H, X = fp.decode(h), fp.decode(x)
    want = hankel.matvec_rows("hankel", H, X, P, rows, processes=8)
    got = fp.decode(y[rows])
    assert got == want


def test_hilbert_n1024_p33220():
    """Configuration of the paper's precision: n = 1024, P = 33220, Hilbert h."""
    need_gpu()
    n, P = 1024, 33220
    h, x = si.hilbert_case(n, P, seed=0)
    announce("fft hilbert", n, P)
    y, rc, flags, err = _oneshot("hankel", h, x, n, P)
    assert rc == 0 and flags == 0
    print("max rounding distance", err, flush=True)
    rows = [0, 1, 511, 1022, 1023]
    _sampled_rows_check(h, x, y, P, rows)
    if kronecker.available():
        assert np.array_equal(y, kronecker.hankel_matvec_words(h, x, P))


def test_index_axis_16384():
    """n > 4096 needs a 16384-point index-axis transform (two 8192-point halves)."""
    need_gpu()
    n, P = 4100, 300
    h = si.uniform(2 * n - 1, P, (68,))
    x = si.uniform(n, P, (69,))
    announce("fft Nt=16384", n, P)
    y, rc, flags, err = _oneshot("hankel", h, x, n, P)
    assert rc == 0 and flags == 0
    rows = [0, 1, 2047, 4098, 4099]
    _sampled_rows_check(h, x, y, P, rows)
    if kronecker.available():
        assert np.array_equal(y, kronecker.hankel_matvec_words(h, x, P))
    yt, rc, _, _ = _oneshot("toeplitz", h, x, n, P)
    assert np.array_equal(yt, y[::-1])


@pytest.mark.parametrize("algo", ["split_fft", "ntt"])
def test_largest_planned_sizes(algo):
    """The largest shapes of the planned paths: n = 8192 (index axis of 16384
    points) at the paper's P, and P = HMV_MAX_P (40960 bits) at n = 4096.
    Sampled rows against the oracle; the Toeplitz product of the same data is
    the Hankel output reversed."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    for n, P in ((8192, 33220), (4096, hmv.MAX_P)):
        h = si.uniform(2 * n - 1, P, (74, n, P))
        x = si.uniform(n, P, (75, n, P))
        announce("fft largest", algo, n, P)
        y, rc, flags, err = _oneshot("hankel", h, x, n, P, algo=algo)
        assert rc == 0 and flags == 0
        _sampled_rows_check(h, x, y, P, [0, 1, n // 2, n - 2, n - 1])
        yt, rc, _, _ = _oneshot("toeplitz", h, x, n, P, algo=algo)
        assert rc == 0 and np.array_equal(yt, y[::-1])


def test_index_axis_8192_ragged_all_kinds():
    """2048 < n < 4096: an 8192-point index axis with a ragged window, every
    kind, against the exact GMP product (and sampled schoolbook rows)."""
    need_gpu()
    n, P = 3001, 700
    h = si.uniform(2 * n - 1, P, (70,))
    x = si.uniform(n, P, (71,))
    announce("fft Nt=8192", n, P)
    y, rc, flags, _ = _oneshot("hankel", h, x, n, P)
    assert rc == 0 and flags == 0
    _sampled_rows_check(h, x, y, P, [0, 1, 1500, 2999, 3000])
    if kronecker.available():
        assert np.array_equal(y, kronecker.hankel_matvec_words(h, x, P))
    yt, rc, _, _ = _oneshot("toeplitz", h, x, n, P)
    assert rc == 0 and np.array_equal(yt, y[::-1])
    c = h[:n].copy()
    yc, rc, _, _ = _oneshot("circulant", c, x, n, P)
    assert rc == 0
    rows = [0, 7, 3000]
    want = hankel.matvec_rows("circulant", fp.decode(c), fp.decode(x), P, rows, processes=8)
    assert fp.decode(yc[rows]) == want


def test_planned_session_equals_exact_product():
    """The planned path at the session shape (n = 4096, P = 33220, unit-norm
    x): two consecutive matvecs on one plan, each equal to the GMP product."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    if not kronecker.available():
        pytest.skip("GMP not available for the full-vector check")
    n, P = 4096, 33220
    h = si.session_h(n, P)
    plan = hmv.Plan("hankel", hmv.to_device(h), n, P, algo="split_fft")
    for k in range(2):
        x = si.session_x(n, P, k)
        announce("fft session", n, P, k)
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        plan.matvec(hmv.to_device(x), y)
        rc, flags, err = hmv.read_status(plan.ws)
        assert rc == 0 and flags == 0 and err < 0.25
        assert np.array_equal(hmv.to_host(y), kronecker.hankel_matvec_words(h, x, P))
    plan.close()


@pytest.mark.parametrize("n,P", [(40, 700), (200, 1500), (300, 2000), (3001, 700), (1000, 33220)])
def test_every_launch_variant_is_exact(n, P):
    """Each launch variant the tuner may pick (radix-16 or radix-8 register
    transforms, XCD-grouped or linear columns) gives the exact words; the
    shapes cover 64-, 256-, 512- and 4096-point index halves and limb
    transforms."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    h = si.uniform(2 * n - 1, P, (72, n))
    x = si.uniform(n, P, (73, n))
    hd, xd = hmv.to_device(h), hmv.to_device(x)
    if n <= 300:
        want = hankel.matvec_words("hankel", h, x, P)
    elif kronecker.available():
        want = kronecker.hankel_matvec_words(h, x, P)
    else:
        pytest.skip("GMP not available for the full-vector check")
    try:
        for cv in range(4):
            for rv in range(2):
                hmv.force_variants(cv, rv)
                plan = hmv.Plan("hankel", hd, n, P, algo="split_fft")
                info = plan.info()
                announce("fft variant", n, P, cv, rv, info["w"], info["Nt"], info["Nz"])
                y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
                plan.matvec(xd, y)
                rc, flags, _ = hmv.read_status(plan.ws)
                assert rc == 0 and flags == 0
                assert np.array_equal(hmv.to_host(y), want), (cv, rv)
                plan.close()
    finally:
        hmv.force_variants(-1, -1)
    hmv.autotune(True)
    plan = hmv.Plan("hankel", hd, n, P, algo="split_fft")
    info = plan.info()
    print("tuned variants", info["cols_variant"], info["rows_inv_variant"], flush=True)
    y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
    plan.matvec(xd, y)
    assert np.array_equal(hmv.to_host(y), want)
    plan.close()


@pytest.mark.parametrize("n,P,expect3", [(33, 1000, False), (200, 1500, False),
                                         (257, 3322, False), (1000, 33220, True)])
def test_every_spectrum_layout_is_exact(n, P, expect3):
    """Each spectrum layout the planner may pick gives the exact words, for
    the three kinds: limb transforms of a power of two or of 3 * 2^k points,
    with the two real limb bins in their own columns or sharing one.  At
    n = 1000, P = 33220 every admissible width has 2L - 1 <= 6144 < 8192, so
    the 3K form is taken there."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    kinds = ("hankel", "toeplitz", "circulant") if n <= 300 else ("hankel",)
    forms = set()
    try:
        for kind in kinds:
            hl = n if kind == "circulant" else 2 * n - 1
            h = si.uniform(hl, P, (74, n, P))
            x = si.uniform(n, P, (75, n, P))
            if n <= 300:
                want = hankel.matvec_words(kind, h, x, P)
            elif kronecker.available():
                want = kronecker.hankel_matvec_words(h, x, P)
            else:
                pytest.skip("GMP not available for the full-vector check")
            hd, xd = hmv.to_device(h), hmv.to_device(x)
            for z3 in (0, 1):
                for pack in (0, 1):
                    hmv.force_layout(z3, pack)
                    plan = hmv.Plan(kind, hd, n, P, algo="split_fft")
                    info = plan.info()
                    Nz = info["Nz"]
                    announce("fft layout", kind, n, P, z3, pack, info["w"], Nz,
                             info["spectrum_cols"])
                    assert info["spectrum_cols"] == Nz // 2 + 1 - pack
                    if z3 == 0:
                        assert Nz & (Nz - 1) == 0
                    forms.add((Nz % 3 == 0, pack))
                    y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
                    plan.matvec(xd, y)
                    rc, flags, err = hmv.read_status(plan.ws)
                    assert rc == 0 and flags == 0 and err < info["bound"]
                    assert np.array_equal(hmv.to_host(y), want), (kind, z3, pack)
                    plan.close()
    finally:
        hmv.force_layout(-1, -1)
    if expect3:
        assert (True, 0) in forms and (True, 1) in forms


@pytest.mark.parametrize("n,P", [(200, 1500), (1000, 33220)])
def test_every_tile_width_is_exact(n, P):
    """Every pair of spectrum tile widths the tuner may pick (2, 4 or 8 bins
    for the spectra of x and of y) gives the exact words, for a 3K and a
    power-of-two limb transform, Hankel and Toeplitz."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    h = si.uniform(2 * n - 1, P, (76, n, P))
    x = si.uniform(n, P, (77, n, P))
    if n <= 300:
        want = hankel.matvec_words("hankel", h, x, P)
    elif kronecker.available():
        want = kronecker.hankel_matvec_words(h, x, P)
    else:
        pytest.skip("GMP not available for the full-vector check")
    hd, xd = hmv.to_device(h), hmv.to_device(x)
    try:
        for z3 in (0, 1):
            for tx in (2, 4, 8):
                for ty in (2, 4, 8):
                    hmv.force_layout(z3, -1)
                    hmv.force_tiles(tx, ty)
                    for kind in ("hankel", "toeplitz"):
                        plan = hmv.Plan(kind, hd, n, P, algo="split_fft")
                        info = plan.info()
                        assert (info["x_tile"], info["y_tile"]) == (tx, ty)
                        announce("fft tiles", kind, n, P, z3, tx, ty, info["Nz"])
                        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
                        plan.matvec(xd, y)
                        rc, flags, _ = hmv.read_status(plan.ws)
                        assert rc == 0 and flags == 0
                        got = hmv.to_host(y)
                        assert np.array_equal(got if kind == "hankel" else got[::-1], want), \
                            (kind, z3, tx, ty)
                        plan.close()
    finally:
        hmv.force_tiles(-1, -1)
        hmv.force_layout(-1, -1)
    plan = hmv.Plan("hankel", hd, n, P, algo="split_fft")
    info = plan.info()
    print("tuned tiles", info["x_tile"], info["y_tile"], "variants", info["cols_variant"],
          info["rows_inv_variant"], flush=True)
    assert info["x_tile"] in (2, 4, 8) and info["y_tile"] in (2, 4, 8)
    plan.close()


def test_graph_captured_planned_step():
    """A planned matvec at the session shape (n = 4096, P = 33220) captured in
    a HIP graph: three replays, each on a different x copied into the
    captured input buffer (with eager work and synchronisations between the
    replays), each equal to the eager result and to the GMP product."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    if not kronecker.available():
        pytest.skip("GMP not available for the full-vector check")
    n, P = 4096, 33220
    h = si.session_h(n, P)
    plan = hmv.Plan("hankel", hmv.to_device(h), n, P, algo="split_fft")
    W = hmv.words(P)
    xs = [si.session_x(n, P, k) for k in (3, 4, 5)]
    xg = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    yg = torch.zeros_like(xg)
    announce("graph capture", n, P)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        xg.copy_(hmv.to_device(xs[0]))
        plan.matvec(xg, yg)                 # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.matvec(xg, yg)
    torch.cuda.synchronize()
    ye = torch.zeros_like(xg)
    for k, x in enumerate(xs):
        announce("graph replay", k)
        xg.copy_(hmv.to_device(x))
        yg.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = hmv.to_host(yg)
        rc, flags, err = hmv.read_status(plan.ws)
        assert rc == 0 and flags == 0 and err < 0.25, k
        plan.matvec(hmv.to_device(x), ye)   # eager, same plan and workspace
        torch.cuda.synchronize()
        assert np.array_equal(got, hmv.to_host(ye)), k
        assert np.array_equal(got, kronecker.hankel_matvec_words(h, x, P)), k
    del g
    plan.close()
