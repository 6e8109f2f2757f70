"""The whole batch in one cooperative launch (hmv_batch_matvec_single):
outputs bit-identical to the oracle on a small mix, to the per-pass
launches on the 256-instance mix, the range flag, and the edge cases (one
instance, n = 1, a member too large for the single launch)."""
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


@pytest.mark.parametrize("specs_seed", [5, 8])
def test_mixed_batch_equals_oracle(specs_seed):
    need_gpu()
    from paper_1402_5287_amd import hmv
    specs = si.batch_instances(60, seed=specs_seed, n_lo=1, n_hi=300,
                               precisions=(64, 200, 1024, 3322))
    host, items = _make(specs, seed=specs_seed)
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_single_workspace_bytes(probs))
    announce("batch single launch", len(specs), specs_seed)
    hmv.batch_matvec_single(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0, flags
    for (kname, h, x), (_, _, _, y, n, P) in zip(host, items):
        assert np.array_equal(hmv.to_host(y), hankel.matvec_words(kname, h, x, P)), (kname, n, P)


@pytest.mark.parametrize("spec", [(0, 1, 64), (1, 1, 3322), (2, 1, 5), (0, 2048, 1024),
                                  (2, 977, 200)])
def test_one_instance(spec):
    need_gpu()
    from paper_1402_5287_amd import hmv
    host, items = _make([spec], seed=9)
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_single_workspace_bytes(probs))
    announce("batch single launch, one instance", spec)
    hmv.batch_matvec_single(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0
    kname, h, x = host[0]
    n, P = spec[1], spec[2]
    got = hmv.to_host(items[0][3])
    if n <= 1000:
        assert np.array_equal(got, hankel.matvec_words(kname, h, x, P))
    else:
        from oracle import fixedpoint as fp
        rows = [0, 1, n // 2, n - 1]
        want = hankel.matvec_rows(kname, fp.decode(h), fp.decode(x), P, rows, processes=2)
        assert fp.decode(got[rows]) == want


def test_range_flag():
    need_gpu()
    from paper_1402_5287_amd import hmv
    from oracle import fixedpoint as fp
    specs = [(0, 40, 1024), (1, 7, 64), (2, 100, 3322)]
    host, items = _make(specs, seed=7)
    kname, h, x = host[1]
    X = fp.decode(x)
    X[3] = (1 << 64) + 1
    bad = list(items)
    bad[1] = (kname, items[1][1], hmv.to_device(fp.encode(X, 64)), items[1][3], 7, 64)
    probs = hmv.batch_problems(bad)
    ws = hmv.workspace(hmv.batch_single_workspace_bytes(probs))
    announce("batch single launch, range")
    hmv.batch_matvec_single(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == hmv.ERANGE and (flags & 1)
    # the other members are still exact
    for j in (0, 2):
        kname, h, x = host[j]
        n, P = specs[j][1], specs[j][2]
        assert np.array_equal(hmv.to_host(items[j][3]), hankel.matvec_words(kname, h, x, P))


def test_full_uneven_batch_of_256_equals_per_pass_launches():
    need_gpu()
    from paper_1402_5287_amd import hmv
    specs = si.batch_instances(256)
    items = []
    for i, (kind, n, P) in enumerate(specs):
        kname = ("hankel", "toeplitz", "circulant")[kind]
        h, x = si.batch_operands(i, kind, n, P)
        y = torch.zeros((n, hmv.words(P)), dtype=torch.int64, device="cuda")
        items.append((kname, hmv.to_device(h), hmv.to_device(x), y, n, P))
    probs = hmv.batch_problems(items)
    ws = hmv.workspace(hmv.batch_single_workspace_bytes(probs))
    announce("batch 256 single launch")
    hmv.batch_matvec_single(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0, flags
    single = [it[3].clone() for it in items]
    for it in items:
        it[3].zero_()
    announce("batch 256 per-pass launches")
    hmv.batch_matvec(probs, ws)
    rc, flags, _ = hmv.read_status(ws)
    assert rc == 0 and flags == 0
    for i, it in enumerate(items):
        assert torch.equal(single[i], it[3]), (i, it[0], it[4], it[5])
