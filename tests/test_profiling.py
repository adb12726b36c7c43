"""Host-side checks of the profile summaries' staleness guard: the recorded
source hash follows the kernel code, not its comments or layout."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1211_0582_amd import profiling  # noqa: E402


def _tree(tmp_path, name, text):
    d = tmp_path / name
    d.mkdir()
    (d / "k.hpp").write_text(text)
    (d / "notes.txt").write_text(name)      # not a source: ignored
    return str(d)


def test_source_hash_ignores_comments_and_whitespace(tmp_path):
    a = _tree(tmp_path, "a", "// header\nint f(int x) { return x + 1; }  /* tail */\n")
    b = _tree(tmp_path, "b", "/* other\n   words */ int f(int x)\n{\n  return x + 1;  // same code\n}\n")
    c = _tree(tmp_path, "c", "int f(int x) { return x + 2; }\n")
    assert profiling.source_hash(a) == profiling.source_hash(b)
    assert profiling.source_hash(a) != profiling.source_hash(c)


def test_committed_traffic_summary_names_the_dominant_kernels():
    path = os.path.join(ROOT, "profiles", "rhs_traffic_k48_n5.txt")
    text = open(path).read()
    assert "source_sha256:" in text
    for kname in ("void dgd::rhs_mfma_kernel<5, float, true, 0, false, 3>(dgd::RhsArgs)",
                  "void dgd::rhs_mfma_kernel<5, float, false, 0, false, 3>(dgd::RhsArgs)"):
        assert "kernel: " + kname in text


def _rows(kind, name, counter, value, dispatch):
    return {"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": str(value), "Dispatch_Id": str(dispatch)}


def test_calibration_picks_the_copy_of_the_stated_size():
    # A run with the 256 MiB calibration copy (dispatch 2) and a larger state
    # copy (dispatch 9): the scale comes from the former.
    kib = 256 * 1024.0
    fetch = [_rows("f", "copyBuffer", "FETCH_SIZE", kib / 2, 2), _rows("f", "copyBuffer", "FETCH_SIZE", 3 * kib / 2, 9)]
    write = [_rows("w", "copyBuffer", "WRITE_SIZE", kib, 2), _rows("w", "copyBuffer", "WRITE_SIZE", 3 * kib, 9)]
    f, w = profiling._calibration_copy(fetch, write, kib)
    assert (f, w) == (kib / 2, kib)
