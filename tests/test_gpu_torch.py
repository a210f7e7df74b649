"""The Hellmann-Feynman backward behind torch.autograd (binding eig_function):
checked in a child process, where torch can be imported before libkth.so."""
import os
import subprocess
import sys

import pytest

from tests.gpu_util import note

pytestmark = pytest.mark.gpu


def test_autograd_function():
    pytest.importorskip("torch")
    script = os.path.join(os.path.dirname(__file__), "torch_autograd_check.py")
    note("autograd function (child process)")
    r = subprocess.run([sys.executable, "-u", script], capture_output=True, text=True, timeout=240)
    print(r.stdout[-3000:], r.stderr[-3000:], flush=True)
    assert r.returncode == 0
    assert "autograd check ok" in r.stdout
