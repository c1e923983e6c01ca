"""The C ABI library loads and exports every function include/msdd.h declares (no GPU needed),
and host-side validation paths that never reach a kernel."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "msdd.h")) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(msdd_[a-z_]+)\s*\(", txt)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["msdd_create", "msdd_setup", "msdd_solve", "msdd_apply", "msdd_stats",
                 "msdd_last_error", "msdd_destroy", "msdd_default_options"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2106_06404_amd import binding as B
    L = B.load()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(B.EXPORTS) <= set(_declared())


def test_default_options_and_profile_names():
    from paper_2106_06404_amd import binding as B
    o = B.default_options()
    assert o.precision == B.MSDD_FP64 and o.block == 16 and o.eig_tol > 0
    L = B.load()
    names = [L.msdd_profile_name(i) for i in range(B.MSDD_NPROF)]
    assert all(n is not None for n in names)
    assert L.msdd_profile_name(B.MSDD_NPROF) is None


def test_create_without_gpu_reports_device_error():
    """Without a GPU (this container) the library reports MSDD_EDEVICE; it never falls back."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2106_06404_amd import binding as B
    with pytest.raises(B.MsddError) as e:
        B.Msdd()
    assert e.value.code == B.MSDD_EDEVICE


def test_null_context_arguments():
    from paper_2106_06404_amd import binding as B
    L = B.load()
    assert L.msdd_setup(None, 1, None, None, None, 1, 1, None, None, 1, None, None, None, None,
                        None, 2, None, 0.1) == B.MSDD_EINVAL
    assert L.msdd_solve(None, None, None, 1e-8, 1, None, None) == B.MSDD_EINVAL
    assert L.msdd_last_error(None) == b"null context"
    L.msdd_destroy(None)
