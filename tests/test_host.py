"""Host-side behaviour that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_binding_has_no_cpu_fallback():
    """Without a GPU the library's context cannot be created: the product
    path raises instead of computing anything on the host."""
    import pytest
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2609_07577_amd import hg
    with pytest.raises(RuntimeError):
        hg.Context(0)


def test_tuning_struct_layout_matches_header():
    """hg_tuning is four int32 fields in the order the header declares."""
    from paper_2609_07577_amd import hg
    assert [f[0] for f in hg.Tuning._fields_] == ["single_pass_load16", "pass_fill16",
                                                  "dense_ratio", "wide_loads"]
    hdr = open(os.path.join(ROOT, "include", "hg.h")).read()
    body = hdr[hdr.index("typedef struct {\n  int32_t single_pass_load16;"):]
    body = body[:body.index("} hg_tuning;")]
    assert body.count("int32_t") == 4
    assert body.index("single_pass_load16") < body.index("pass_fill16") < \
        body.index("dense_ratio") < body.index("wide_loads")
