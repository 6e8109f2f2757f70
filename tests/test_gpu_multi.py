"""Blocks of vectors with one plan, Y = A [x_1 .. x_k] (hmv_plan_matvec_multi):
every output equals the single-vector planned product, the oracle at small
sizes and the exact GMP product at the session shape (n = 4096, P = 33220)."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import fixedpoint as fp, hankel, kronecker
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _block(plan, xs):
    """(outputs of the block call, outputs of k single calls, status, max error)."""
    from paper_1402_5287_amd import hmv
    k, n, W = len(xs), plan.n, hmv.words(plan.P)
    xd = hmv.to_device(np.concatenate(xs, axis=0))
    y = torch.full((k * n, W), -1, dtype=torch.int64, device="cuda")
    ws = plan.multi_workspace(k)
    plan.matvec_multi(xd, y, k, ws)
    rc, flags, err = hmv.read_status(ws)
    singles = []
    for j in range(k):
        yj = torch.zeros((n, W), dtype=torch.int64, device="cuda")
        plan.matvec(xd[j * n:(j + 1) * n], yj)
        singles.append(hmv.to_host(yj))
    torch.cuda.synchronize()
    return hmv.to_host(y).reshape(k, n, W), singles, rc, flags, err


@pytest.mark.parametrize("kind,n,P,algo,k", [
    ("hankel", 64, 3322, "split_fft", 3), ("toeplitz", 200, 1500, "split_fft", 2),
    ("circulant", 77, 1000, "split_fft", 5), ("toeplitz", 300, 2000, "split_fft", 4),
    ("hankel", 1, 100, "split_fft", 2), ("circulant", 100, 2000, "ntt", 3),
    ("toeplitz", 90, 1500, "karatsuba", 2)])
def test_block_equals_single_and_oracle(kind, n, P, algo, k):
    need_gpu()
    from paper_1402_5287_amd import hmv
    hl = n if kind == "circulant" else 2 * n - 1
    h = si.uniform(hl, P, (80, n, P))
    xs = [si.uniform(n, P, (81, n, P, j)) for j in range(k)]
    plan = hmv.Plan(kind, hmv.to_device(h), n, P, algo=algo)
    announce("multi", kind, n, P, algo, k, plan.info()["Nz"])
    Y, singles, rc, flags, _ = _block(plan, xs)
    assert rc == hmv.OK and flags == 0
    H = fp.decode(h)
    for j in range(k):
        assert np.array_equal(Y[j], singles[j]), j
        want = fp.encode(hankel.matvec_ints(kind, H, fp.decode(xs[j]), P), P)
        assert np.array_equal(Y[j], want), j
    plan.close()


def test_every_variant_and_layout_in_blocks():
    """The launch variants and spectrum layouts at a 3K shape, k = 3."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P, k = 300, 2000, 3
    h = si.uniform(2 * n - 1, P, (82,))
    xs = [si.uniform(n, P, (83, j)) for j in range(k)]
    want = [fp.encode(hankel.matvec_ints("toeplitz", fp.decode(h), fp.decode(x), P), P)
            for x in xs]
    try:
        for cv in range(4):
            for z3, pack in ((0, 0), (1, 1), (1, 0)):
                hmv.force_variants(cv, 0)
                hmv.force_layout(z3, pack)
                plan = hmv.Plan("toeplitz", hmv.to_device(h), n, P, algo="split_fft")
                announce("multi variant", cv, z3, pack, plan.info()["Nz"])
                Y, _, rc, flags, _ = _block(plan, xs)
                assert rc == hmv.OK and flags == 0
                for j in range(k):
                    assert np.array_equal(Y[j], want[j]), (cv, z3, pack, j)
                plan.close()
    finally:
        hmv.force_variants(-1, -1)
        hmv.force_layout(-1, -1)


@pytest.mark.parametrize("k", [2, 4])
def test_session_shape_block_equals_gmp(k):
    """n = 4096, P = 33220, unit-norm x: a block of k equals k single products
    bit for bit, and the exact GMP product on two of its vectors."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    if not kronecker.available():
        pytest.skip("GMP not available for the full-vector check")
    n, P = 4096, 33220
    h = si.session_h(n, P)
    plan = hmv.Plan("hankel", hmv.to_device(h), n, P, algo="split_fft")
    xs = [si.session_x(n, P, 10 * k + j) for j in range(k)]
    announce("multi session", n, P, k)
    Y, singles, rc, flags, err = _block(plan, xs)
    assert rc == hmv.OK and flags == 0 and err < 0.25
    for j in range(k):
        assert np.array_equal(Y[j], singles[j]), j
    for j in (0, k - 1):
        assert np.array_equal(Y[j], kronecker.hankel_matvec_words(h, xs[j], P)), j
    plan.close()


def test_block_argument_checks():
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 32, 500
    h = si.uniform(2 * n - 1, P, (84,))
    plan = hmv.Plan("hankel", hmv.to_device(h), n, P, algo="split_fft")
    W = hmv.words(P)
    x = torch.zeros((2 * n, W), dtype=torch.int64, device="cuda")
    y = torch.zeros_like(x)
    ws = plan.multi_workspace(2)
    assert plan.matvec_multi(x, y, 0, ws, check=False) == hmv.EINVAL
    assert plan.matvec_multi(x, y, 65, ws, check=False) == hmv.EINVAL
    small = plan.multi_workspace(1)
    assert plan.matvec_multi(x, y, 2, small, check=False) == hmv.ENOMEM
    assert hmv.lib().hmv_plan_multi_workspace_bytes(plan.handle, 0) == hmv.EINVAL
    plan.close()
