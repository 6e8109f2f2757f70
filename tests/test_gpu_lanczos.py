"""Lanczos tridiagonalisation on the GPU (hmv_lanczos) against the fixed-point
oracle (oracle/lanczos.py): alphas, betas and the basis bit for bit, on
small Hankel matrices, the closed forms, several paths and the paper's
precision."""
import pytest

import seeded_inputs as si
from oracle import fixedpoint as fp, lanczos
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _unit_start(n, P, seed):
    return si.unit_norm(si.uniform(n, P, seed), P)


def _run(H, q1, n, P, steps, algo="split_fft"):
    from paper_1402_5287_amd import hmv
    plan = hmv.Plan("hankel", hmv.to_device(fp.encode(H, P)), n, P, algo=algo)
    alpha, beta, done, basis, ws = plan.lanczos(hmv.to_device(fp.encode(q1, P)), steps,
                                                basis=True)
    rc, flags, _ = hmv.read_status(ws)
    k = int(done.item())
    out = (fp.decode(hmv.to_host(alpha[:k])), fp.decode(hmv.to_host(beta[:k])),
           [fp.decode(hmv.to_host(basis[j])) for j in range(k)])
    plan.close()
    return out, rc, flags


@pytest.mark.parametrize("n,P,steps,algo", [
    (8, 100, 8, "split_fft"), (16, 3322, 12, "split_fft"), (33, 1000, 20, "ntt"),
    (24, 500, 10, "karatsuba"), (64, 3322, 16, "split_fft"), (5, 64, 5, "auto"),
    # 512 entries and more: one work-group per entry for the dot products and the
    # updates (fewer entries split every product over several work-groups); past
    # 1024 entries a dot-product work-group takes several entries
    (600, 200, 3, "split_fft"), (1100, 100, 2, "split_fft")])
def test_equals_oracle(n, P, steps, algo):
    need_gpu()
    H = fp.decode(si.uniform(2 * n - 1, P, (100, n, P)))
    q1 = fp.decode(_unit_start(n, P, (101, n, P)))
    announce("lanczos", n, P, steps, algo)
    (a, b, basis), rc, flags = _run(H, q1, n, P, steps, algo)
    assert rc == 0 and flags == 0
    wa, wb, wbasis = lanczos.lanczos(H, q1, P, steps)
    assert len(a) == len(wa)
    assert a == wa
    assert b == wb
    assert basis == wbasis


@pytest.mark.parametrize("P", [3, 64, 3322])
def test_closed_forms(P):
    need_gpu()
    # exchange matrix from e_0: alpha = 0, 0; beta = 1, 0 (stop after 2)
    n = 4
    H = [0] * (2 * n - 1)
    H[n - 1] = 1 << P
    q1 = [1 << P, 0, 0, 0]
    announce("lanczos exchange", P)
    (a, b, _), rc, _ = _run(H, q1, n, P, 6)
    assert rc == 0 and a == [0, 0] and b == [1 << P, 0]
    # rank one, h = 1/2, n = 5: alpha = 1/2, 2; beta = 1, 0
    n, half = 5, 1 << (P - 1)
    H = [half] * (2 * n - 1)
    q1 = [1 << P] + [0] * (n - 1)
    announce("lanczos rank one", P)
    (a, b, basis), rc, _ = _run(H, q1, n, P, 6)
    assert rc == 0 and a == [half, 2 << P] and b == [1 << P, 0]
    assert basis[1] == [0, half, half, half, half]


def test_paper_precision():
    """n = 100 (the paper's Lanczos sizes), P = 33220 bits, 4 steps."""
    need_gpu()
    n, P, steps = 100, 33220, 4
    H = fp.decode(si.uniform(2 * n - 1, P, (102,)))
    q1 = fp.decode(_unit_start(n, P, (103,)))
    announce("lanczos paper precision", n, P, steps)
    (a, b, basis), rc, flags = _run(H, q1, n, P, steps)
    assert rc == 0 and flags == 0
    wa, wb, wbasis = lanczos.lanczos(H, q1, P, steps)
    assert a == wa and b == wb and basis == wbasis


def test_toeplitz_plan_is_refused():
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 8, 100
    h = si.uniform(2 * n - 1, P, (104,))
    plan = hmv.Plan("toeplitz", hmv.to_device(h), n, P, algo="split_fft")
    with pytest.raises(hmv.HmvError) as ei:
        plan.lanczos(hmv.to_device(_unit_start(n, P, (105,))), 3)
    assert ei.value.code == hmv.EINVAL
    plan.close()
