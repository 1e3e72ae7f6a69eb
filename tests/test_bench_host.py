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


def _summary(tmp_path, src_hash, numbering="curve"):
    prof = tmp_path / "profiles"
    prof.mkdir()
    lines = [f"kernel_source_sha256_16: {src_hash}", f"numbering: {numbering}", ""]
    for i, k in enumerate(bench.LAUNCHES_PER_STEP):
        lines.append(f"{k:14s} 20  1.0  1.0  hbm_bytes_per_launch={(i + 1) * 1e9:.4e}  "
                     f"alg_bytes_per_launch=1.0e+09  1.0  1.0  1.00")
    (prof / "dycore_fp64_r2b8x90_hbm_counters.txt").write_text("\n".join(lines) + "\n")


def test_counted_traffic_only_from_a_summary_of_the_same_code(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _summary(tmp_path, "00112233aabbccdd")
    kinds = list(bench.LAUNCHES_PER_STEP)
    col = kinds.index("column_corr") + 1
    assert bench.measured_traffic("column_corr", "00112233aabbccdd", "fp64") == col * 1e9
    assert bench.measured_traffic("column_corr", "ffffffffffffffff", "fp64") is None
    assert bench.measured_traffic("column_corr", "00112233aabbccdd", "fp64", numbering="hilbert") is None
    assert bench.measured_traffic("column_corr", "00112233aabbccdd", "mixed") is None
    # a whole step: every kernel's bytes x its launches per substep x substeps
    want = sum((i + 1) * 1e9 * n for i, n in enumerate(bench.LAUNCHES_PER_STEP.values())) * 5
    assert bench.step_traffic("00112233aabbccdd", "fp64", 5) == want
    assert bench.step_traffic("ffffffffffffffff", "fp64", 5) is None


def test_step_accounting_against_the_peak():
    out = bench.step_accounting(1e10, "fp64", counted_b=1000.0)
    for basis, b in bench.STEP_BUDGET_B["fp64"].items():
        assert out[basis]["B_per_cell_level_substep"] == b
        assert abs(out[basis]["frac"] - b * 1e10 / (bench.HBM_PEAK_GBS * 1e9)) < 1e-4
    assert out["counted"]["GBs"] == 10000.0
    assert abs(out["counted"]["frac"] - 10000.0 / bench.HBM_PEAK_GBS) < 1e-4
