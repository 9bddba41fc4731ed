"""Host-side checks of the C ABI that need no GPU: the shared library loads,
exports every function include/ccake.h declares, and rejects bad
configurations in ccake_workspace_bytes (a pure host call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "ccake.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccake_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_2511_22852_amd import binding as B
    L = B.lib()
    names = header_functions()
    assert len(names) >= 26
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing
    assert sorted(names) == sorted(B.EXPORTS)


@pytest.mark.parametrize("field,value", [("dim", 4), ("coords", 7), ("ncharge", 2), ("h", -1.0),
                                         ("precision", 3), ("density_mode", 5)])
def test_workspace_bytes_rejects_bad_config(field, value):
    from paper_2511_22852_amd import binding as B
    cfg = B.config()
    setattr(cfg, field, value)
    nb = ctypes.c_size_t()
    assert B.lib().ccake_workspace_bytes(ctypes.byref(cfg), 100, ctypes.byref(nb)) == B.E_ARG


def test_workspace_bytes_grows_with_n():
    from paper_2511_22852_amd import binding as B
    cfg = B.config(viscous=True, eta_over_s=0.08, ncharge=3)
    sizes = []
    for n in (1, 1000, 40000):
        nb = ctypes.c_size_t()
        assert B.lib().ccake_workspace_bytes(ctypes.byref(cfg), n, ctypes.byref(nb)) == B.OK
        sizes.append(nb.value)
    assert sizes[0] < sizes[1] < sizes[2]
    # about 2 kB per particle: state and stage copies, neighbour records, sums,
    # row caches and the diffusion records and sums
    assert sizes[2] < 2500 * 40000
    # 3+1D adds the skin list that the pair passes after a step's first
    # density pass walk: 4096 two-byte entries per particle
    cfg3 = B.config(dim=3, viscous=True, eta_over_s=0.08, ncharge=3)
    nb3 = ctypes.c_size_t()
    assert B.lib().ccake_workspace_bytes(ctypes.byref(cfg3), 40000, ctypes.byref(nb3)) == B.OK
    assert 8192 * 40000 <= nb3.value - sizes[2] < (8192 + 1500) * 40000
    bad = B.config(viscous=True, eta_over_s=0.0)
    assert B.lib().ccake_workspace_bytes(ctypes.byref(bad), 10, ctypes.byref(nb)) == B.E_ARG
