"""The oracle and the GPU library share no code: neither side imports,
includes or links the other (CPU only)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _files(sub, exts):
    for dp, _, fs in os.walk(os.path.join(ROOT, sub)):
        for f in fs:
            if f.endswith(exts):
                yield os.path.join(dp, f)


def test_oracle_does_not_use_library():
    for f in _files("oracle", (".py", ".c", ".h")):
        text = open(f).read()
        assert not re.search(r"^\s*(import|from)\s+paper_2508_12093_amd", text, re.M), f
        assert "libppstat" not in text and "ppstat.h" not in text, f


def test_library_does_not_use_oracle():
    pat = re.compile(r"\boracle\b|ckks_ref|orc_")
    for f in _files("paper_2508_12093_amd", (".py", ".cpp", ".hip", ".h", ".hpp")):
        text = open(f).read()
        assert not pat.search(text), f
    for f in _files("include", (".h",)):
        assert not pat.search(open(f).read()), f
