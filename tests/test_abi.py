"""The C-ABI libraries load and export what their headers declare (no GPU)."""
import ctypes
import os
import re

from paper_1402_3325_amd import sakura

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_hip_library_exports_every_declared_symbol():
    names = sakura.declared_functions()
    assert {"sakura_create", "sakura_destroy", "sakura_step", "sakura_evolve",
            "sakura_energy", "sakura_last_error"} <= set(names)
    L = ctypes.CDLL(sakura.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_stats_struct_matches_header():
    text = open(sakura.HEADER).read()
    body = text[text.index("typedef struct {\n    uint64_t pair_solves"):]
    body = body[:body.index("} sakura_stats;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(\w+)(?:\[\d+\])?;", body)
    assert fields == [f for f, _ in sakura.Stats._fields_]
    body = text[text.index("typedef struct {\n    int guess"):]
    body = re.sub(r"/\*.*?\*/", "", body[:body.index("} sakura_opts;")], flags=re.S)
    assert re.findall(r"\b(\w+);", body) == [f for f, _ in sakura.Opts._fields_]


def test_oracle_library_exports_every_declared_symbol(oracle):
    text = open(os.path.join(ROOT, "oracle", "sakura_oracle.h")).read()
    names = sorted(set(re.findall(r"\b(sref_[a-z0-9_]+)\s*\(", text)))
    L = oracle.lib()
    assert not [n for n in names if not hasattr(L, n)]


def test_product_path_never_loads_the_oracle():
    """The HIP binding and kernels neither import nor link the oracle."""
    pkg = os.path.join(ROOT, "paper_1402_3325_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "sref_" not in src, f


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of every struct in include/sakura.h, as gcc lays
    them out, against the ctypes mirrors of the binding."""
    import subprocess
    fields = {"sakura_opts": sakura.Opts, "sakura_stats": sakura.Stats,
              "sakura_guess_model": sakura.GuessModel, "sakura_fit_opts": sakura.FitOpts}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sakura.h"', "int main(void) {"]
    for cname, py in fields.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, py in fields.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_enum_constants_match_the_header():
    """The binding's scheme, starter and status constants are the header's."""
    text = open(sakura.HEADER).read()
    for name, value in (("SAKURA_SCHEME_PSI", sakura.SCHEME_PSI),
                        ("SAKURA_SCHEME_UNMERGED", sakura.SCHEME_UNMERGED),
                        ("SAKURA_SCHEME_TRIPLE_JUMP", sakura.SCHEME_TRIPLE_JUMP),
                        ("SAKURA_GUESS_LEARNED", sakura.GUESS_LEARNED),
                        ("SAKURA_ENOMODEL", sakura.ENOMODEL)):
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == value, name


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr and not r.stdout
