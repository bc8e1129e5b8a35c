"""The C-ABI library loads and exports every function include/zpl.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import re
from pathlib import Path

ROOT = Path(__file__).resolve().parent.parent


def declared_functions():
    text = (ROOT / "include" / "zpl.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(zpl_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1305_6738_amd import zpl
    assert zpl.LIB_PATH.exists(), "libzpl.so not built"
    lib = ctypes.CDLL(str(zpl.LIB_PATH))
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(zpl.exported_symbols())


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1305_6738_amd import zpl
    monkeypatch.setattr(zpl, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(zpl, "_lib", None)
    try:
        zpl.lib()
    except RuntimeError as e:
        assert "no CPU fallback" in str(e)
    else:
        raise AssertionError("expected a RuntimeError")


def test_bench_refuses_multi_gpu():
    import bench
    assert bench.main(["--gpus", "2"]) == 2
