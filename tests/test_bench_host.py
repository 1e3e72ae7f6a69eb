"""Host-side helpers of bench.py (no GPU): the identity of the kernel code
that decides whether a committed counter summary still describes it."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_code_tokens_drop_comments_and_layout():
    a = 'int x = 1;  // one\n/* block\n comment */ double  y =\n  "a // b /* c */";\n'
    b = "int x = 1; double y = \"a // b /* c */\";"
    assert bench._code_tokens(a) == b
    assert bench._code_tokens("char q = '\"'; // \"\nint z;") == "char q = '\"'; int z;"


def test_code_tokens_see_code_changes():
    base = "a = b * c; // product"
    assert bench._code_tokens(base) != bench._code_tokens("a = b + c; // product")
    assert bench._code_tokens(base) == bench._code_tokens("a  =  b *\n c;   // the product")


def test_kernel_source_hash_is_stable():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
