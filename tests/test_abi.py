"""The C ABI library loads on the host and exports every entry point that
include/cnmf.h declares; argument checks that need no GPU reject bad calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cnmf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cnmf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_1812_04315_amd as cnmf
    if not os.path.exists(cnmf.LIB_PATH):
        pytest.fail("libcnmf.so is not built: run __graft_entry__.build()")
    return cnmf.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    import paper_1812_04315_amd as cnmf
    assert sorted(cnmf.EXPORTED) == _declared()


def test_null_context_and_bad_arguments(lib):
    import paper_1812_04315_amd as cnmf
    assert lib.cnmf_sweep_right(None, 1, 1, None, 1, 1, None, 1, 0, None, 1) == cnmf.EINVAL
    assert lib.cnmf_sweep_left(None, 1, 1, None, 1, 1, None, 1, None, 1, 0) == cnmf.EINVAL
    assert lib.cnmf_sweep_dual(None, 1, 1, None, 1, 1, None, 1, None, 1, None, 1, None, 1,
                               0) == cnmf.EINVAL
    assert lib.cnmf_sweep_dual_bf16(None, 1, 1, None, 1, 1, None, 1, None, 1, None, 1, None, 1,
                                    0) == cnmf.EINVAL
    assert lib.cnmf_orth(None, 4, 2, None, None, 0, 1e-9, None, None) == cnmf.EINVAL
    assert lib.cnmf_lipschitz(None, 3, None, None) == cnmf.EINVAL
    prm = cnmf.params(5)
    assert lib.cnmf_rsi(None, 10, 10, None, 10, ctypes.byref(prm), None, None, None, None,
                        None, None) == cnmf.EINVAL
    assert lib.cnmf_solve(None, 0, 10, 10, None, 10, None, None, None, None,
                          ctypes.byref(prm), None, None, None, None) == cnmf.EINVAL
    assert lib.cnmf_status(None, None) == cnmf.EINVAL
    assert lib.cnmf_destroy(None) == cnmf.EINVAL
    out = ctypes.c_void_p()
    assert lib.cnmf_create(None, 0, None) == cnmf.EINVAL


def test_params_default(lib):
    import paper_1812_04315_amd as cnmf
    p = cnmf.Params()
    lib.cnmf_params_default(ctypes.byref(p))
    assert (p.nu, p.q, p.inner_max, p.inner_min) == (10, 4, 500, 1)
    assert p.inner_ratio == 1e-3 and p.tau2 == 1e-9
    assert lib.cnmf_strerror(cnmf.EINVAL) == b"invalid argument"


def test_product_path_has_no_fallback(monkeypatch):
    """Without the built library every entry point raises; nothing computes
    on the host."""
    import paper_1812_04315_amd as cnmf
    monkeypatch.setattr(cnmf, "_lib", None)
    monkeypatch.setattr(cnmf, "LIB_PATH", "/nonexistent/libcnmf.so")
    with pytest.raises(RuntimeError):
        cnmf.lib()


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1812_04315_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
