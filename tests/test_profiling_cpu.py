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


def test_pmc_filter_keeps_only_dispatches_that_reach_the_minimum(tmp_path):
    from paper_0912_3824_amd.profiling import pmc
    rows = ["Dispatch_Id,Kernel_Name,Grid_Size,Counter_Name,Counter_Value"]
    for did, (waves, valu) in enumerate([(10, 5.0), (5000, 100.0), (6000, 300.0)]):
        rows += [f"{did},k_build,64,SQ_WAVES,{waves}", f"{did},k_build,64,SQ_INSTS_VALU,{valu}"]
    (tmp_path / "run_counter_collection.csv").write_text("\n".join(rows) + "\n")
    every = pmc(str(tmp_path)).splitlines()
    busy = pmc(str(tmp_path), ("SQ_WAVES", 1000)).splitlines()
    assert "k_build | 64 | SQ_INSTS_VALU | 3 | 135" in every
    assert "k_build | 64 | SQ_INSTS_VALU | 2 | 200" in busy
    assert "k_build | 64 | SQ_WAVES | 2 | 5500" in busy
