"""Host-side checks that the product path and the CPU oracle stay apart.

The oracle is test infrastructure: the HIP library and its Python binding
must neither import, link nor call it, and the oracle must not reuse the
library's code.  Only the seeded input generators (synth) serve both.  The
binding must also fail loudly, never fall back, when the library is missing.
"""
import os
import re
import subprocess
import sys

import pytest

from paper_2203_17119_amd import dwf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2203_17119_amd")
ORACLE = os.path.join(ROOT, "oracle")


def _sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(dwf, "_lib", None)
    with pytest.raises(ImportError, match="missing"):
        dwf.load(str(tmp_path / "libdwf.so"))


def test_package_sources_never_reach_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle\b|from\s+\.\.\s*oracle|#\s*include\s*[<\"].*oracle)"
                     r"|liboracle|\bor_[a-z0-9_]+\s*\(", re.M)
    hits = []
    for path in _sources(PKG, (".py", ".cpp", ".hip", ".inl", ".h")):
        for m in pat.finditer(open(path, encoding="utf-8").read()):
            hits.append(f"{os.path.relpath(path, ROOT)}: {m.group(0).strip()}")
    assert not hits, hits


def test_oracle_sources_never_reach_the_library():
    pat = re.compile(r"^\s*(from|import)\s+paper_2203_17119_amd\.(?!synth\b)\w+|libdwf|dwf_common|dwf_internal"
                     r"|#\s*include\s*\".*dwf", re.M)
    hits = []
    for path in _sources(ORACLE, (".py", ".c", ".h")):
        for m in pat.finditer(open(path, encoding="utf-8").read()):
            hits.append(f"{os.path.relpath(path, ROOT)}: {m.group(0).strip()}")
    assert not hits, hits


def test_built_library_does_not_link_the_oracle():
    if not os.path.exists(dwf.LIB_PATH):
        pytest.fail("libdwf.so is not built: run __graft_entry__.build()")
    blob = open(dwf.LIB_PATH, "rb").read()
    assert b"liboracle" not in blob
    for sym in (b"or_hop", b"or_d5", b"or_dirichlet", b"or_gamma"):
        assert sym not in blob, sym


def test_loading_the_library_leaves_the_oracle_unimported():
    code = ("import sys\n"
            "from paper_2203_17119_amd import dwf, synth\n"
            "import paper_2203_17119_amd.rational\n"
            "dwf.load()\n"
            "assert dwf.dwf_abi_version() == 1\n"
            "bad = sorted(m for m in sys.modules if m == 'oracle' or m.startswith('oracle.'))\n"
            "assert not bad, bad\n"
            "print('isolated')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "isolated" in r.stdout
