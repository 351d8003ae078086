"""The C-ABI library loads and exports every symbol include/tnrg.h declares;
host-side logic (layout arithmetic, argument validation, workspace sizing)
works without a GPU (no compute call is made)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tnrg.h")


@pytest.fixture(scope="module")
def lib():
    from conftest import ensure_library
    return ctypes.CDLL(ensure_library())


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("mps_evolve", "mps_overlap", "grape_fidelity_grad"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_symbol(lib):
    from paper_2603_03639_amd import tnrg
    assert set(declared_functions()) == set(tnrg.EXPORTS)


def cap(N, dcap, b):
    return min(dcap, 2 ** b, 2 ** (N - b))


@pytest.mark.parametrize("N,dcap", [(2, 1), (8, 16), (50, 16), (50, 64), (30, 128), (7, 3)])
def test_layout_arithmetic(lib, N, dcap):
    from paper_2603_03639_amd import tnrg
    off = 0
    for j in range(N):
        assert tnrg.site_offset(N, dcap, j) == off
        assert tnrg.bond_cap(N, dcap, j) == cap(N, dcap, j)
        off += cap(N, dcap, j) * 2 * cap(N, dcap, j + 1)
    assert tnrg.traj_elems(N, dcap) == off
    assert tnrg.bond_cap(N, dcap, N) == 1


def test_argument_validation_without_gpu():
    from paper_2603_03639_amd import tnrg
    m = tnrg.Model(N=1, M=5, dt=0.1, chi=4).c()
    rc = tnrg._lib.grape_fidelity_grad(ctypes.byref(m), None, None, None, 1, None, 1, None, None,
                                       0, 0, None, None, None, None, None, None, None, 0, None)
    assert rc == tnrg.EINVAL
    assert b"n = 1" in tnrg._lib.tnrg_last_error()
    m = tnrg.Model(N=8, M=5, dt=0.1, chi=4, zz_mask=np.zeros(7), xt_mask=np.ones(7)).c()
    rc = tnrg._lib.mps_overlap(None, None, None, None, 0, None)
    assert rc == tnrg.EINVAL
    fake = ctypes.c_void_p(0x1000)
    b = tnrg._Batch(2, 8, 4, 0x1000, 0x2000)
    rc = tnrg._lib.grape_fidelity_grad(ctypes.byref(m), fake, fake, fake, 3, fake, 2,
                                       ctypes.byref(b), ctypes.byref(b), 0, 0, fake, fake, fake,
                                       fake, None, None, fake, 16, None)
    assert rc == tnrg.ENOMEM
    bad = tnrg.Model(N=8, M=5, dt=float("nan"), chi=4, zz_mask=np.zeros(7), xt_mask=np.ones(7)).c()
    rc = tnrg._lib.mps_evolve(ctypes.byref(bad), fake, fake, fake, fake, 0, 5, 0, ctypes.byref(b),
                              fake, 1 << 30, None)
    assert rc == tnrg.EINVAL


def test_workspace_bytes_monotone():
    from paper_2603_03639_amd import tnrg
    m = tnrg.Model(N=50, M=200, dt=0.05, chi=64, zz_mask=np.zeros(49), xt_mask=np.ones(49))
    a = tnrg.grape_workspace_bytes(m, 128, 8, 16)
    b = tnrg.grape_workspace_bytes(m, 128, 8, 32)
    c = tnrg.grape_workspace_bytes(m, 128, 8, 16, ckpt_stride=1)
    assert 0 < a < b
    assert c > a            # stride 1 stores every slice
    assert a < 40 * 2 ** 30  # the headline workload fits easily in 288 GB
