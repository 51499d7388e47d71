"""C-ABI library: it loads, exports every symbol include/ck.h declares, and its host-only paths work.

No compute call is made here (no GPU in the build container)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ck.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ck_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1608_05794_amd import ck
    if not os.path.exists(ck.LIB_PATH):
        from paper_1608_05794_amd import build
        build.build()
    return ck.lib()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    from paper_1608_05794_amd import ck
    assert sorted(ck.EXPORTS) == names


def test_host_only_paths(lib, tmp_path):
    from paper_1608_05794_amd import ck
    o = ck.Opts()
    lib.ck_opts_default(C.byref(o))
    assert o.rtol == 1e-8 and o.atol == 1e-12 and o.max_steps == 1000000 and o.refine_sweeps == 3
    assert lib.ck_strerror(-3) == b"malformed mechanism file"
    h = C.c_void_p()
    assert lib.ck_mechanism_load(str(tmp_path / "missing.ckm").encode(), 0, C.byref(h)) == -2
    bad = tmp_path / "bad.ckm"
    bad.write_text("CKMECH 1\nCONST 8.314 101325\nELEMENTS 1\nE H 0.001\nSPECIES 1\nS H oops\n")
    assert lib.ck_mechanism_load(str(bad).encode(), 0, C.byref(h)) == -3
    assert lib.ck_mechanism_load(None, 0, C.byref(h)) == -1
    # argument validation happens before any device work
    assert lib.ck_rhs_eval(None, 1, None, 1, None, None, None) == -1
    assert lib.ck_integrate_ros4(None, 1, None, 1, None, None, None, None, None, None, None, None, None, None) == -1


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    from paper_1608_05794_amd import ck
    monkeypatch.setattr(ck, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(ck, "_lib", None)
    with pytest.raises(ck.CkError):
        ck.lib()


def test_binding_vector_checks():
    """The binding's per-reactor vector checks (host tensors stand in for device ones here)."""
    import torch

    from paper_1608_05794_amd import ck
    cpu = torch.device("cpu")
    v = torch.zeros(8, dtype=torch.float64)
    assert ck._vec(v, 8, cpu, "p") is v
    assert ck._vec(None, 8, cpu, "t") is None
    with pytest.raises(ck.CkError):
        ck._vec(v, 9, cpu, "p")                               # too short
    with pytest.raises(ck.CkError):
        ck._vec(v.to(torch.float32), 8, cpu, "p")             # wrong dtype
    with pytest.raises(ck.CkError):
        ck._vec(torch.zeros(16, dtype=torch.float64)[::2], 8, cpu, "p")   # strided
    with pytest.raises(ck.CkError):
        ck._vec(torch.zeros(2, 8, dtype=torch.float64), 8, cpu, "p")      # not a vector
