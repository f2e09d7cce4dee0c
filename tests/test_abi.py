"""The C-ABI library loads and exports every entry point of include/lprdem.h
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lprdem.h")
LIB = os.path.join(ROOT, "paper_2501_05300_amd", "liblprdem.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:lpr_status|const char\*)\s+(lpr_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("lpr_bed_create", "lpr_step", "lpr_read_contacts", "lpr_read_forces", "lpr_read_reaction"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_lists_every_declared_symbol():
    from paper_2501_05300_amd import lprdem
    assert sorted(lprdem.SYMBOLS) == declared()


def test_binding_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from paper_2501_05300_amd import beds, lprdem
    spec = beds.two_layer_bed(0)
    with pytest.raises(RuntimeError):
        lprdem.Bed(spec)


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs one GPU; --gpus above 1 exits with a message before
    touching a device."""
    import json
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=root)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]
