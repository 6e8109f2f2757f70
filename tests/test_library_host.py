"""Host-side checks of libhmv (no GPU): exported symbols, size queries,
argument validation, the error bound and the root tables."""
import ctypes
import math
import os
import re
from fractions import Fraction

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hmv.h")


def _lib():
    from paper_1402_5287_amd import hmv
    try:
        return hmv, hmv.lib()
    except ImportError as e:
        pytest.skip(str(e))


def test_every_declared_symbol_is_exported():
    hmv, L = _lib()
    text = open(HEADER).read()
    names = set(re.findall(r"\b(hmv_[a-z0-9_]+)\s*\(", text))
    assert len(names) >= 10
    for name in sorted(names):
        assert hasattr(L, name), name
        assert name in hmv.SIGNATURES, f"binding lacks {name}"


def test_words_and_validation():
    hmv, L = _lib()
    assert L.hmv_words(1) == 2 and L.hmv_words(64) == 2 and L.hmv_words(65) == 3
    assert L.hmv_words(33220) == 521 and L.hmv_words(3322) == 53
    assert L.hmv_words(0) == -1 and L.hmv_words(40961) == -1
    # bad arguments are rejected before any device work
    assert L.hmv_hankel_matvec(None, None, None, 4, 64, 0, None, 0, None) == -1
    assert L.hmv_oneshot_workspace_bytes(7, 4, 64, 0) == -1
    assert L.hmv_oneshot_workspace_bytes(0, 0, 64, 0) == -1
    assert L.hmv_plan_bytes(0, 4, 0, 1) == -1
    assert L.hmv_plan_matvec(None, None, None, None, 0, None) == -1
    assert L.hmv_strerror(-2) == b"input magnitude exceeds 1"


def test_size_queries():
    hmv, L = _lib()
    # headline shape: the sizes cover every candidate width; at P = 33220
    # widths 9 and 10 need N_z = 8192 (N_t = 8192): 4097 resident columns,
    # and 4096 spectrum columns per row of x and of y
    n = 4096
    pb = L.hmv_plan_bytes(0, n, 33220, 1)
    assert pb >= 8192 * 4097 * 16
    ws = L.hmv_workspace_bytes(0, n, 33220, 1)
    assert ws >= 2 * 4096 * 4096 * 16
    assert L.hmv_oneshot_workspace_bytes(0, 64, 3322, 4) > 0


def test_planned_paths_size_limit():
    """The planned paths take n up to 8192 (index axis of 16384 points); larger
    n up to HMV_MAX_N is refused with HMV_EUNSUPPORTED, except by the
    schoolbook, which takes every n up to HMV_MAX_N."""
    hmv, L = _lib()
    for algo in (0, 1, 2, 3):
        assert L.hmv_oneshot_workspace_bytes(0, 8192, 3322, algo) > 0
        assert L.hmv_oneshot_workspace_bytes(0, 8193, 3322, algo) == hmv.EUNSUPPORTED
        assert L.hmv_plan_bytes(0, 8193, 3322, algo) == hmv.EUNSUPPORTED
    assert L.hmv_words(hmv.MAX_P) > 0 and L.hmv_words(hmv.MAX_P + 1) == hmv.EINVAL
    assert L.hmv_oneshot_workspace_bytes(0, hmv.MAX_N, 3322, 4) > 0
    assert L.hmv_oneshot_workspace_bytes(0, hmv.MAX_N + 1, 3322, 4) == hmv.EINVAL


def _percival(na, nb, k, beta):
    """Independent evaluation with exact rationals for the powers and a
    rigorous upper rounding of the result."""
    eps = Fraction(1, 2**53)
    s5 = Fraction(2236067977499790, 10**15)   # > sqrt(5)
    f = (1 + eps) ** (3 * k) * (1 + eps * s5) ** (3 * k + 1) * (1 + Fraction(beta)) ** (3 * k) - 1
    return float(Fraction(na) * Fraction(nb) * f)


def test_error_bound_matches_exact_evaluation():
    hmv, L = _lib()
    beta = L.hmv_twiddle_beta()
    assert 0 < beta < 2.0**-52
    for na, nb, k in ((1.0, 1.0, 10), (2.9e6, 3.6e6, 28), (1e5, 2e5, 16), (7.0, 3.0, 1)):
        got = L.hmv_fft_error_bound(na, nb, k, beta)
        want = _percival(na, nb, k, beta)
        assert want <= got <= want * (1 + 1e-5)
    # the naive evaluation loses the 2^-53 terms entirely; ours must not
    assert L.hmv_fft_error_bound(1.0, 1.0, 26, 0.0) > 26 * 3 * 2.0**-53


def test_twiddle_beta_against_mpmath():
    mpmath = pytest.importorskip("mpmath")
    hmv, L = _lib()
    beta = L.hmv_twiddle_beta()
    # beta must dominate the error of correctly rounded roots (about 2^-53.5)
    with mpmath.workprec(200):
        worst = mpmath.mpf(0)
        for N in (16, 256, 4096, 16384):
            for m in range(0, N, max(1, N // 97)):
                c = mpmath.cos(2 * mpmath.pi * m / N)
                s = -mpmath.sin(2 * mpmath.pi * m / N)
                err = abs(mpmath.mpc(float(c), float(s)) - mpmath.mpc(c, s))
                worst = max(worst, err)
    assert float(worst) <= beta


def test_debug_switches_validate_and_restore():
    hmv, L = _lib()
    assert L.hmv_debug_force_layout(2, 0) == hmv.EINVAL
    assert L.hmv_debug_force_layout(0, -2) == hmv.EINVAL
    assert L.hmv_debug_force_layout(0, 1) == 0
    assert L.hmv_debug_force_layout(-1, -1) == 0
    assert L.hmv_debug_force_variants(4, 0) == hmv.EINVAL
    assert L.hmv_debug_force_variants(0, 2) == hmv.EINVAL
    assert L.hmv_debug_force_variants(-1, -1) == 0
    for bad in ((3, 4), (16, -1), (0, 1)):
        assert L.hmv_debug_force_tiles(*bad) == hmv.EINVAL, bad
    assert L.hmv_debug_force_tiles(8, 2) == 0
    assert L.hmv_debug_force_tiles(-1, -1) == 0


def test_single_launch_batch_validation():
    """The one-launch batch checks its arguments before any device work: bad
    lists give HMV_EINVAL, a missing or short workspace HMV_ENOMEM (so the
    256-instance mix has a power-of-two layout, which needs more workspace
    than the per-pass driver's)."""
    import seeded_inputs as si
    hmv, L = _lib()
    fake = 1 << 20                                 # never dereferenced on these paths
    mix = si.batch_instances(256)
    arr = (hmv.Problem * len(mix))()
    for k, (kind, n, P) in enumerate(mix):
        arr[k] = hmv.Problem(kind, P, n, fake, fake, fake)
    ptr = ctypes.cast(arr, ctypes.c_void_p)
    ws = L.hmv_batch_single_workspace_bytes(ptr, len(mix))
    assert ws > L.hmv_batch_workspace_bytes(ptr, len(mix)) > 0
    assert L.hmv_batch_matvec_single(ptr, len(mix), None, 0, None) == hmv.ENOMEM
    assert L.hmv_batch_matvec_single(ptr, len(mix), ctypes.c_void_p(fake), ws - 1,
                                     None) == hmv.ENOMEM
    assert L.hmv_batch_matvec(ptr, len(mix), None, 0, None) == hmv.ENOMEM
    assert L.hmv_batch_matvec_single(None, 3, None, 0, None) == hmv.EINVAL
    assert L.hmv_batch_matvec_single(ptr, 0, None, 0, None) == hmv.EINVAL
    bad = (hmv.Problem * 2)()
    bad[0] = hmv.Problem(0, 64, 4, fake, fake, fake)
    bad[1] = hmv.Problem(0, 64, 4, fake, 0, fake)           # null x
    assert L.hmv_batch_matvec_single(ctypes.cast(bad, ctypes.c_void_p), 2, None, 0,
                                     None) == hmv.EINVAL
    bad[1] = hmv.Problem(0, 64, 4096, fake, fake, fake)     # n above the batch limit
    assert L.hmv_batch_matvec_single(ctypes.cast(bad, ctypes.c_void_p), 2, None, 0,
                                     None) == hmv.EINVAL
