"""The C-ABI library loads without a GPU and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    syms = set()
    for name in os.listdir(os.path.join(ROOT, "include")):
        if not name.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", name)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        syms |= set(re.findall(r"\b(start_[a-z_0-9]+)\s*\(", text))
    return syms


def test_header_declares_the_calls():
    syms = declared_symbols()
    for required in ("start_build_source_tree", "start_build_gas_grid", "start_compute_rates"):
        assert required in syms


def test_library_exports_every_declared_symbol():
    import paper_1005_5312_amd as S
    lib = S.lib()
    missing = [s for s in sorted(declared_symbols()) if not hasattr(lib, s)]
    assert not missing, missing
    assert set(S.EXPORTS) == declared_symbols()


def test_estimate_bytes_monotone():
    import paper_1005_5312_amd as S
    a = S.estimate_bytes(1 << 14, 64, 1 << 14, 5)
    b = S.estimate_bytes(1 << 20, 1 << 20, 1 << 20, 7)
    assert 0 < a < b


def test_binding_refuses_without_gpu():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_1005_5312_amd as S
    with pytest.raises(RuntimeError):
        S.Context(0)
