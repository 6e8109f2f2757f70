"""Floating-point interface (hmv_fplan_*) on the GPU against the floating
oracle: every output significand and exponent equal, for the three kinds,
wide exponent spreads, cancellation to zero, ties, and the range checks."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import fixedpoint as fp, floatio
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _draw(count, P, spread, seed, zeros=0.0):
    """Significands uniform on (-2^P, 2^P), exponents uniform in a window of
    `spread` below a seeded top; a fraction `zeros` of exact zeros."""
    rng = np.random.default_rng(seed)
    M = fp.decode(si.uniform(count, P - 1, seed))          # |M| <= 2^(P-1)
    M = [m * 2 + int(rng.integers(0, 2)) if abs(m * 2) < (1 << P) - 1 else m for m in M]
    top = int(rng.integers(-200, 200))
    e = [top - int(rng.integers(0, spread + 1)) for _ in range(count)]
    for k in range(count):
        if rng.random() < zeros:
            M[k], e[k] = 0, 0
    return M, e


def _run(kind, Mh, eh, Mx, ex, n, P, spread):
    from paper_1402_5287_amd import hmv
    W = hmv.words(P)
    hs = hmv.to_device(fp.encode(Mh, P))
    he = torch.tensor(eh, dtype=torch.int32, device="cuda")
    xs = hmv.to_device(fp.encode(Mx, P))
    xe = torch.tensor(ex, dtype=torch.int32, device="cuda")
    plan = hmv.FPlan(kind, hs, he, n, P, spread)
    ys = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    ye = torch.zeros(n, dtype=torch.int32, device="cuda")
    plan.matvec(xs, xe, ys, ye)
    rc, flags, _ = hmv.read_status(plan.ws)
    got = (fp.decode(hmv.to_host(ys)), ye.cpu().tolist())
    info = plan.info()
    plan.close()
    return got, rc, flags, info


@pytest.mark.parametrize("kind,n,P,spread", [
    ("hankel", 1, 2, 0), ("hankel", 5, 64, 10), ("toeplitz", 33, 65, 100),
    ("circulant", 40, 200, 300), ("hankel", 100, 1000, 64), ("toeplitz", 257, 3322, 700),
    ("hankel", 300, 128, 5000)])
def test_equals_float_oracle(kind, n, P, spread):
    need_gpu()
    hl = n if kind == "circulant" else 2 * n - 1
    Mh, eh = _draw(hl, P, spread, (90, n, P, spread), zeros=0.1)
    Mx, ex = _draw(n, P, spread, (91, n, P, spread), zeros=0.1)
    announce("float", kind, n, P, spread)
    got, rc, flags, info = _run(kind, Mh, eh, Mx, ex, n, P, spread)
    assert rc == 0 and flags == 0, (rc, flags)
    assert info["Q"] == P + spread
    want = floatio.matvec(kind, Mh, eh, Mx, ex, P)
    assert got[0] == want[0]
    assert got[1] == want[1]
    for m in got[0]:
        assert m == 0 or (1 << (P - 1)) <= abs(m) < (1 << P)


def test_cancellation_ties_and_powers_of_two():
    need_gpu()
    P = 4
    # y_0: 3 * 5 * 2^(5+2-8) - 6 * 5 * 2^(4+2-8) = 0; y_1: a tie (23 -> 24)
    Mh, eh = [3, -6, 4], [5, 4, -3]
    Mx, ex = [5, 5], [2, 2]
    announce("float hand cases")
    got, rc, _, _ = _run("hankel", Mh, eh, Mx, ex, 2, P, 16)
    assert rc == 0
    assert got == floatio.matvec("hankel", Mh, eh, Mx, ex, P)
    assert (got[0][0], got[1][0]) == (0, 0)
    # all significands at the extremes, equal exponents
    P, n = 65, 6
    lim = (1 << P) - 1
    Mh = [lim if k % 2 else -lim for k in range(2 * n - 1)]
    Mx = [-lim, lim, lim, -lim, lim, lim]
    got, rc, _, _ = _run("hankel", Mh, [7] * len(Mh), Mx, [-3] * n, n, P, 0)
    assert rc == 0
    assert got == floatio.matvec("hankel", Mh, [7] * len(Mh), Mx, [-3] * n, P)


def test_paper_precision_n1024():
    """P = 33220 significant bits, n = 1024, exponents spread over 40 bits."""
    need_gpu()
    n, P, spread = 1024, 33220, 40
    Mh, eh = _draw(2 * n - 1, P, spread, (92,))
    Mx, ex = _draw(n, P, spread, (93,))
    announce("float paper precision", n, P)
    got, rc, flags, info = _run("hankel", Mh, eh, Mx, ex, n, P, spread)
    assert rc == 0 and flags == 0
    print("inner plan", info["algo"], info["w"], info["Nz"], flush=True)
    rows = [0, 1, 511, 1023]
    H, Fh = floatio.aligned_ints(Mh, eh)
    X, Fx = floatio.aligned_ints(Mx, ex)
    S = [sum(H[i + j] * X[j] for j in range(n)) for i in rows]   # eq. (1), sampled rows
    for r, s in zip(rows, S):
        m, e = floatio.round_significant(s, Fh + Fx - 2 * P, P)
        assert (got[0][r], got[1][r]) == (m, e), r


def test_range_errors():
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 8, 100
    Mh, eh = _draw(2 * n - 1, P, 10, (94,))
    Mx, ex = _draw(n, P, 10, (95,))
    # h wider than the spread: refused at plan time
    Mh[3] = Mh[3] or 1
    eh_wide = list(eh)
    eh_wide[3] = max(eh) + 50
    with pytest.raises(hmv.HmvError) as ei:
        _run("hankel", Mh, eh_wide, Mx, ex, n, P, 20)
    assert ei.value.code == hmv.ERANGE
    # a significand with P + 1 bits: refused
    Mh2 = list(Mh)
    Mh2[0] = 1 << P
    with pytest.raises(hmv.HmvError) as ei:
        _run("hankel", Mh2, eh, Mx, ex, n, P, 20)
    assert ei.value.code == hmv.ERANGE
    # x wider than the spread: flagged on the device
    ex_wide = list(ex)
    Mx[2] = Mx[2] or 1
    ex_wide[2] = max(ex) - 40
    announce("float range flag")
    _, rc, flags, _ = _run("hankel", Mh, eh, Mx, ex_wide, n, P, 20)
    assert rc == hmv.ERANGE and flags & 1
