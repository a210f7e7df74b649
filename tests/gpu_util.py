"""Shared helpers of the GPU tests (which run through the C ABI of libkth.so)."""
import sys

import numpy as np


def note(msg: str):
    """Print and flush the case about to run on the GPU."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def kth():
    import paper_1710_05134_amd as K
    K.lib()
    return K
