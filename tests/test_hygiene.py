"""The oracle is test infrastructure and independent of the HIP path: no product source imports,
includes or links anything under oracle/, and the oracle imports nothing of the product; only the
seeded input generators (phantoms/) serve both, and they hold none of the method's arithmetic."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _files(top, exts):
    for d, _, names in os.walk(os.path.join(ROOT, top)):
        if "__pycache__" in d or "_build" in d:
            continue
        for n in names:
            if n.endswith(exts):
                yield os.path.join(d, n)


def test_product_does_not_use_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle|#\s*include\s*[<\"].*oracle)", re.M)
    hits = [f for f in _files("paper_2605_19737_amd", (".py", ".hip", ".hpp", ".h", ".cpp")) if pat.search(open(f).read())]
    hits += [f for f in _files("include", (".h",)) if pat.search(open(f).read())]
    assert not hits, hits


def test_oracle_does_not_use_the_product():
    pat = re.compile(r"(paper_2605_19737_amd|libdvr\.so|\bdvr\.h|csrc)")
    hits = [f for f in _files("oracle", (".py", ".c", ".h")) if pat.search(open(f).read())]
    assert not hits, hits


def test_inputs_module_holds_no_method_arithmetic():
    """phantoms/ builds volumes, TFs and cameras; it imports neither the product nor the oracle and
    defines no function of the method's steps (features, eigenvalues, raymarch, compositing)."""
    src = "".join(open(f).read() for f in _files("phantoms", (".py",)))
    assert not re.search(r"^\s*(import|from)\s+(oracle|paper_2605_19737_amd)", src, re.M)
    defs = re.findall(r"^\s*def\s+(\w+)", src, re.M)
    bad = [d for d in defs if re.search(r"frangi|vessel|hessian|eig|raymarch|composit|curvature|trilinear", d, re.I)]
    assert defs and not bad, bad
    assert "eigvalsh" not in src and "linalg.eig" not in src


def test_only_tests_bench_and_smoke_touch_the_oracle():
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle)", re.M)
    users = set()
    for f in _files(".", (".py",)):
        rel = os.path.relpath(f, ROOT)
        if rel.startswith(("oracle" + os.sep, "_work" + os.sep, "gpurun_out" + os.sep)):
            continue
        if pat.search(open(f).read()):
            users.add(rel.split(os.sep)[0] if os.sep in rel else rel)
    assert users <= {"tests", "bench.py", "__graft_entry__.py"}, users
