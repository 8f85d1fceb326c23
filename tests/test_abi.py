"""The C-ABI library loads and exports every entry point include/em.h declares
(no compute calls: this runs without a GPU)."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "em.h")).read()
    return sorted(set(re.findall(r"\b(em_[a-z_0-9]+)\s*\(", txt)))


def test_header_matches_binding_list():
    from paper_2604_10743_amd._binding import API
    assert sorted(API) == _declared()


def test_library_exports_every_symbol():
    import paper_2604_10743_amd as P
    L = P.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_no_cpu_fallback_in_package():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_2604_10743_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("Oracle", "").lower() or f == "synth.py", f
