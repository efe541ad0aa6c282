"""Host-side helpers of the profile summaries (no GPU)."""
from paper_0912_3824_amd.profiling import _code_only, kernel_source_hash


def test_comments_are_dropped_and_literals_kept():
    src = 'int a = 1; // note\n/* block\n comment */ const char *s = "// kept /* too */";\nchar q = \'"\'; int b;'
    assert _code_only(src) == 'int a = 1; const char *s = "// kept /* too */"; char q = \'"\'; int b;'


def test_hash_ignores_comments_and_layout_but_not_code():
    files = {"step.hip": "int f() {\n  return 1; // one\n}\n", "dev_common.hpp": "", "md_dev.hpp": "",
             "ds.hpp": "", "kernels.hpp": ""}
    base = kernel_source_hash(files.get)
    files["step.hip"] = "/* the function */ int f() { return 1; }"
    assert kernel_source_hash(files.get) == base
    files["step.hip"] = "int f() { return 2; }"
    assert kernel_source_hash(files.get) != base
