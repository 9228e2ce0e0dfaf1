"""Host-side checks of bench.py's source fingerprint, which decides whether
the committed hardware-counter traffic still describes the PCG kernels:
comments and layout must not change it, code must."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_comments_and_layout_are_ignored():
    a = "int f(int x) {\n  return x + 1; // add one\n}\n"
    b = "/* a helper */\nint f(int x)\n{\n    return x + 1;   /* add\n one */\n}"
    assert bench._code_text(a) == bench._code_text(b)


def test_code_changes_are_seen():
    a = "int f(int x) { return x + 1; }"
    b = "int f(int x) { return x + 2; }"
    assert bench._code_text(a) != bench._code_text(b)


def test_comment_markers_inside_literals_are_code():
    s = 'const char* u = "a // b /* c */"; char q = \'"\'; int k; // gone'
    assert bench._code_text(s) == 'const char* u = "a // b /* c */"; char q = \'"\'; int k;'


def test_fingerprint_is_stable():
    assert bench.source_fingerprint() == bench.source_fingerprint()
    assert len(bench.source_fingerprint()) == 16
