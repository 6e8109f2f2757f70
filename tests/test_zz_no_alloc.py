"""The allocation-free planned matvec (hmv_plan_matvec_noalloc) against the
planned matvec with a caller workspace (hmv_plan_matvec), through the C ABI:
bit-equal outputs on consecutive calls of shrinking size, status reporting,
and the refusal of a plan whose workspace exceeds the fixed scratch."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import fixedpoint as fp, hankel
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _plan(kind, n, P, algo, seed):
    from paper_1402_5287_amd import hmv
    hl = n if kind == "circulant" else 2 * n - 1
    h = si.uniform(hl, P, (70, seed, n, P))
    return h, hmv.Plan(kind, hmv.to_device(h), n, P, algo=algo)


def _both(plan, x_np, status):
    """(y from hmv_plan_matvec, y from hmv_plan_matvec_noalloc, status of the latter)."""
    from paper_1402_5287_amd import hmv
    W = hmv.words(plan.P)
    xd = hmv.to_device(x_np)
    y_ref = torch.zeros((plan.n, W), dtype=torch.int64, device="cuda")
    y_na = torch.full((plan.n, W), -1, dtype=torch.int64, device="cuda")
    plan.matvec(xd, y_ref)
    status.fill_(0x55)                     # stale bytes the call must overwrite
    plan.matvec_noalloc(xd, y_na, status=status)
    rc, flags, err = hmv.read_status(status)
    return hmv.to_host(y_ref), hmv.to_host(y_na), rc, flags, err


def test_noalloc_equals_workspace_path_on_shrinking_calls():
    need_gpu()
    from paper_1402_5287_amd import hmv
    status = torch.zeros(256, dtype=torch.uint8, device="cuda")
    # a large call first (its spectra fill much of the fixed scratch), then
    # smaller ones of other kinds, paths and sizes, then the large one again
    cases = [("hankel", 1024, 33220, "split_fft", 0), ("toeplitz", 200, 3322, "split_fft", 1),
             ("circulant", 77, 1000, "auto", 2), ("hankel", 100, 2000, "ntt", 3),
             ("toeplitz", 90, 1500, "karatsuba", 4), ("hankel", 1024, 33220, "split_fft", 5)]
    plans = {}
    for kind, n, P, algo, seed in cases:
        key = (kind, n, P, algo)
        if key not in plans:
            plans[key] = _plan(kind, n, P, algo, len(plans))
        h, plan = plans[key]
        x = si.uniform(n, P, (71, seed, n, P))
        announce("noalloc", kind, n, P, algo, seed)
        y_ref, y_na, rc, flags, err = _both(plan, x, status)
        assert rc == hmv.OK and flags == 0, (kind, n, P, algo, rc, flags)
        assert np.array_equal(y_na, y_ref), (kind, n, P, algo)
        if plan.info()["algo"] == hmv.SPLIT_FFT:
            assert err <= plan.info()["bound"]
        if n <= 200:
            want = fp.encode(hankel.matvec_ints(kind, fp.decode(h), fp.decode(x), P), P)
            assert np.array_equal(y_na, want), (kind, n, P, algo)
    for _, plan in plans.values():
        plan.close()


def test_noalloc_without_status_buffer_and_range_flag():
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 64, 3322
    h, plan = _plan("hankel", n, P, "split_fft", 9)
    W = hmv.words(P)
    x = si.uniform(n, P, (72, n, P))
    y_ref = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    y_na = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    announce("noalloc no status", n, P)
    plan.matvec(hmv.to_device(x), y_ref)
    plan.matvec_noalloc(hmv.to_device(x), y_na)          # status stays in the fixed array
    torch.cuda.synchronize()
    assert np.array_equal(hmv.to_host(y_na), hmv.to_host(y_ref))
    # an input of magnitude above 1 is flagged in the caller's status buffer
    X = fp.decode(x)
    X[5] = (1 << P) + 1
    bad = fp.encode(X, P)
    status = torch.zeros(256, dtype=torch.uint8, device="cuda")
    announce("noalloc range flag", n, P)
    plan.matvec_noalloc(hmv.to_device(bad), y_na, status=status)
    rc, flags, _ = hmv.read_status(status)
    assert rc == hmv.ERANGE and flags & 1
    # and the next good call clears it
    plan.matvec_noalloc(hmv.to_device(x), y_na, status=status)
    rc, flags, _ = hmv.read_status(status)
    assert rc == hmv.OK and flags == 0
    assert np.array_equal(hmv.to_host(y_na), hmv.to_host(y_ref))
    plan.close()


def test_noalloc_refuses_a_plan_beyond_the_fixed_scratch():
    need_gpu()
    from paper_1402_5287_amd import hmv
    n, P = 6000, 33220
    h, plan = _plan("hankel", n, P, "split_fft", 10)
    need = plan.info()["matvec_workspace_bytes"]
    limit = 448 << 20
    assert need > limit
    W = hmv.words(P)
    x = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    y = torch.zeros((n, W), dtype=torch.int64, device="cuda")
    announce("noalloc refusal", n, P, need)
    rc = plan.matvec_noalloc(x, y, check=False)
    assert rc == hmv.ENOMEM
    assert b"fixed scratch" in hmv.lib().hmv_last_error()
    plan.close()
    # null arguments are refused before any device work
    assert hmv.lib().hmv_plan_matvec_noalloc(None, None, None, None, None) == hmv.EINVAL
