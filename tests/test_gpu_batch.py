"""Batched launches: many uneven (kind, n, P) products, one launch per pass
and transform size, each product checked against the oracle."""
import numpy as np
import pytest

import seeded_inputs as si
from oracle import hankel
from tests.gpu_util import announce, need_gpu, torch

pytestmark = pytest.mark.gpu


def _make(specs, seed):
    from paper_1402_5287_amd import hmv
    host, items = [], []
    for i, (kind, n, P) in enumerate(specs):
        kname = ("hankel", "toeplitz", "circulant")[kind]
        h, x = si.batch_operands(i, kind, n, P, seed=seed)
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        items.append((kname, hmv.to_device(h), hmv.to_device(x), y, n, P))
        host.append((kname, h, x))
    return host, items


def test_mixed_batch_bit_exact():
    need_gpu()
    from paper_1402_5287_amd import hmv
    specs = si.batch_instances(60, seed=5, n_lo=1, n_hi=300, precisions=(64, 200, 1024, 3322))
    host, items = _make(specs, seed=5)
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_workspace_bytes(probs))
    announce("batch", len(specs))
    hmv.batch_matvec(probs, ws)
    rc, flags, err = hmv.read_status(ws)
    assert rc == 0 and flags == 0, flags
    for (kname, h, x), (_, _, _, y, n, P) in zip(host, items):
        assert np.array_equal(hmv.to_host(y), hankel.matvec_words(kname, h, x, P)), (kname, n, P)


def test_batch_equals_single_paths_at_paper_sizes():
    """A batch with paper-sized members: every output equals the planned
    single-instance split-FFT path (itself pinned to the oracle)."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    specs = si.batch_instances(24, seed=6)
    host, items = _make(specs, seed=6)
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_workspace_bytes(probs))
    announce("batch paper sizes", len(specs))
    hmv.batch_matvec(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0
    for (kname, h, x), (_, hd, xd, y, n, P) in zip(host, items):
        y1 = torch.zeros_like(y)
        hmv.matvec(kname, hd, xd, y1, n, P, algo="split_fft")
        assert torch.equal(y, y1), (kname, n, P)
    # and a few members against the oracle directly
    for (kname, h, x), (_, _, _, y, n, P) in list(zip(host, items))[:3]:
        if n <= 200:
            assert np.array_equal(hmv.to_host(y), hankel.matvec_words(kname, h, x, P))


def test_batch_out_of_range_flag():
    """One member with an x entry just outside [-1, 1] sets the range flag of
    the batch; the batch without it is clean."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    from oracle import fixedpoint as fp
    specs = [(0, 40, 1024), (1, 7, 64), (2, 100, 3322)]
    host, items = _make(specs, seed=7)
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_workspace_bytes(probs))
    announce("batch range ok")
    hmv.batch_matvec(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0
    kname, h, x = host[1]
    X = fp.decode(x)
    X[3] = (1 << 64) + 1
    bad = list(items)
    bad[1] = (kname, items[1][1], hmv.to_device(fp.encode(X, 64)), items[1][3], 7, 64)
    probs = hmv.batch_problems(bad)
    announce("batch range bad")
    hmv.batch_matvec(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == hmv.ERANGE and (flags & 1)


@pytest.mark.skip(reason="exercises the single-launch work-queue batch driver, which is switched "
                         "off: its launch did not finish on two GPU runs (the second after a "
                         "change to its fences) and the cause has not been established")
def test_batch_spin_limit_exit_path():
    """With a tiny spin limit the dependency waits give up: the launch still
    completes (every wave exits) and reports the spin flag or a valid result."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    specs = [(0, 200, 1024)] * 8
    host, items = _make(specs, seed=7)
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_workspace_bytes(probs))
    hmv.set_batch_spin_limit(1)
    try:
        hmv.batch_matvec(probs, ws)
        rc, flags, _ = hmv.read_status(ws)
    finally:
        hmv.set_batch_spin_limit(0)
    assert rc == 0
    if not flags & 4:
        for (kname, h, x), (_, _, _, y, n, P) in zip(host, items):
            assert np.array_equal(hmv.to_host(y), hankel.matvec_words(kname, h, x, P))


def test_full_uneven_batch_of_256():
    """The whole 256-instance mix (n log-uniform in 32..2048, P from {1024,
    4096, 16384, 33220}, a third of each kind) in one batched call: every
    product equals the single-product path, and a sample of members equals
    the oracle (plain sums where small, the GMP product for Hankel members,
    sampled rows otherwise)."""
    need_gpu()
    from paper_1402_5287_amd import hmv
    specs = si.batch_instances(256)
    host, items = [], []
    for i, (kind, n, P) in enumerate(specs):
        kname = ("hankel", "toeplitz", "circulant")[kind]
        h, x = si.batch_operands(i, kind, n, P)
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        items.append((kname, hmv.to_device(h), hmv.to_device(x), y, n, P))
        host.append((kname, h, x))
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_workspace_bytes(probs))
    announce("batch 256", hmv.batch_launches(probs), "launches")
    hmv.batch_matvec(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0, flags
    single_ws = hmv.workspace(max(hmv.oneshot_workspace_bytes(k, n, P)
                                  for (k, _, _, _, n, P) in items))
    for i, (kname, hd, xd, y, n, P) in enumerate(items):
        y1 = torch.zeros_like(y)
        hmv.matvec(kname, hd, xd, y1, n, P, ws=single_ws)
        torch.cuda.synchronize()
        assert torch.equal(y1, y), (i, kname, n, P)
    from oracle import fixedpoint as fp, kronecker
    for i in range(0, 256, 16):
        kname, h, x = host[i]
        n, P = items[i][4], items[i][5]
        got = hmv.to_host(items[i][3])
        if n * n * P <= 300 * 300 * 1024:
            assert np.array_equal(got, hankel.matvec_words(kname, h, x, P)), i
        elif kname == "hankel" and kronecker.available():
            assert np.array_equal(got, kronecker.hankel_matvec_words(h, x, P)), i
        else:
            rows = [0, n // 2, n - 1]
            want = hankel.matvec_rows(kname, fp.decode(h), fp.decode(x), P, rows, processes=3)
            assert fp.decode(got[rows]) == want, i
