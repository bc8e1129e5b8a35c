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


# Every struct of the C ABI and its ctypes mirror in the binding.
def _mirrors():
    from paper_1305_6738_amd import zpl
    return {"zpl_cell": zpl.Cell, "zpl_sim_opts": zpl.SimOpts, "zpl_tune_entry": zpl.TuneEntry,
            "zpl_serve_opts": zpl.ServeOpts, "zpl_serve_result": zpl.ServeResult}


def test_header_struct_layouts_match_the_binding(tmp_path):
    """A C program compiled against include/zpl.h prints sizeof and offsetof
    of every field of every ABI struct; the ctypes mirrors in zpl.py must lay
    out the same bytes (a drift would otherwise surface only on the GPU)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    assert cc, "no C compiler"
    mirrors = _mirrors()
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "zpl.h"', "int main(void) {"]
    for name, cls in mirrors.items():
        lines.append('  printf("%s sizeof %%zu\\n", sizeof(%s));' % (name, name))
        for f in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, f[0], name, f[0]))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", str(ROOT / "include"), str(src),
                    "-o", str(exe)], check=True, capture_output=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        struct, field, value = line.split()
        got[(struct, field)] = int(value)
    for name, cls in mirrors.items():
        assert got[(name, "sizeof")] == ctypes.sizeof(cls), name
        for f in cls._fields_:
            assert got[(name, f[0])] == getattr(cls, f[0]).offset, (name, f[0])
    # and the header declares no ABI struct without a mirror
    text = (ROOT / "include" / "zpl.h").read_text()
    declared = set(re.findall(r"typedef struct (zpl_[a-z_]+) \{", text))
    assert declared == set(mirrors), declared ^ set(mirrors)


def test_plan_forms_from_c(tmp_path):
    """The host-only planner called from C through the shared library: the
    built-in rule (no tuning table) gives the lane form to a light cell, the
    wave form to one whose values above 48 are many, and the heavy form to a
    heavy tail (Sect. 3 cells of different shapes), with ZPL_EINVAL for an
    exponent outside [1.01, 64]."""
    import shutil
    import subprocess
    from paper_1305_6738_amd import zpl
    cc = shutil.which("gcc") or shutil.which("cc")
    src = tmp_path / "plan.c"
    src.write_text(r'''
#include <stdio.h>
#include "zpl.h"
int main(void) {
  zpl_cell cells[3] = {{3.0, 100, 1000, 1, 0, 0, 0}, {1.6, 1000, 1000, 1, 1, 0, 0},
                       {1.2, 100000, 1000, 1, 2, 0, 0}};
  int32_t forms[3] = {0, 0, 0};
  zpl_status st = zpl_plan_forms(NULL, 0, cells, 3, forms);
  printf("%d %d %d %d\n", (int)st, forms[0], forms[1], forms[2]);
  cells[0].alpha = 0.5;
  st = zpl_plan_forms(NULL, 0, cells, 3, forms);
  printf("%d\n", (int)st);
  return 0;
}
''')
    exe = tmp_path / "plan"
    libdir = zpl.LIB_PATH.parent
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", str(ROOT / "include"), str(src),
                    "-L", str(libdir), "-l:libzpl.so", "-Wl,-rpath," + str(libdir), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out[:4] == ["0", str(zpl.FORM_LANE), str(zpl.FORM_WAVE), str(zpl.FORM_HEAVY)], out
    assert out[4] == str(-1), out
