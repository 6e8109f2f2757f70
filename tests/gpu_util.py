"""Helpers for the GPU tests (device plumbing only)."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def announce(*parts):
    """Print what names the case before a GPU step (flushed)."""
    print("[case]", *parts, flush=True)
    sys.stdout.flush()
