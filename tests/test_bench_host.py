"""Host-side logic of bench.py (no GPU): the code fingerprint that ties a
committed HBM-traffic record to the kernel source it was measured on, and the
records themselves."""
import importlib.util
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_fingerprint_ignores_comments_and_white_space_only(tmp_path):
    b = _bench()
    base = "int f(int x)\n{\n    return x + 1;   // one more\n}\n/* block\n   comment */\n"
    same = "// a new first line\nint f(int x) {\n  return x + 1;\n}\n"
    other = "int f(int x)\n{\n    return x + 2;   // one more\n}\n"
    paths = []
    for i, text in enumerate((base, same, other)):
        p = tmp_path / f"k{i}.hip"
        p.write_text(text)
        paths.append(str(p))
    f0, f1, f2 = (b.code_fingerprint(p) for p in paths)
    assert f0 == f1
    assert f0 != f2
    assert len(f0) == 16


def test_traffic_records_parse():
    """Every kernel of the committed traffic summaries has a calibrated record
    (the value bench.py reports, or None once the kernel's code changes)."""
    b = _bench()
    for kernel, tag in (("k_adj_fac", "mixed_lmax2500"), ("k_triple_bt", "mixed_lmax2500"),
                        ("k_adj_fac64", "fp64_lmax2500"), ("k_triple_f64", "fp64_lmax2500")):
        path = os.path.join(ROOT, "profiles", f"{tag}_hbm_traffic.txt")
        lines = [l.split() for l in open(path)]
        assert any(f[:1] == ["calibration"] for f in lines), tag
        rec = [f for f in lines if f[:2] == ["traffic", kernel]]
        assert len(rec) == 1 and len(rec[0]) == 6, (kernel, rec)
        v = b.measured_traffic(kernel, tag)
        assert v is None or v > 0
