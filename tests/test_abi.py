"""The C-ABI library loads and exports every symbol declared in include/frg.h;
host-side argument checks and the host geometry (no device needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1510_07799_amd import frg, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "frg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(frg_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(frg.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(frg.SIGNATURES) == set(names)


def test_status_strings():
    L = frg.lib()
    for st in range(6):
        assert L.frg_status_str(st)
    assert L.frg_status_str(99) == b"unknown status"


@pytest.mark.parametrize("bad", [dict(N=10), dict(N=0), dict(N=260), dict(n_rad=0),
                                 dict(t=0.0), dict(mu=float("nan")), dict(U=float("inf"))])
def test_bad_parameters_rejected_on_host(bad):
    p = dict(t=1.0, tp=0.0, mu=0.0, U=2.0, N=16, n_rad=8, n_ang=8)
    p.update(bad)
    with pytest.raises(frg.FRGError) as e:
        frg.host_tables(**p)
    assert e.value.status == frg.EINVAL
    pp = frg.params(**p)
    h = ctypes.c_void_p()
    assert frg.lib().frg_create(ctypes.byref(pp), ctypes.byref(h)) == frg.EINVAL
    assert not h.value


def test_too_many_points_not_supported():
    with pytest.raises(frg.FRGError) as e:
        frg.host_tables(N=8, n_rad=64, n_ang=32)
    assert e.value.status == frg.ENOTSUP


def test_null_arguments():
    L = frg.lib()
    assert L.frg_create(None, None) == frg.EINVAL
    assert L.frg_rhs(None, 0.1, None, None, 0, None) == frg.EINVAL
    assert L.frg_sizes(None, None, None, None, None) == frg.EINVAL
    assert L.frg_destroy(None) == frg.OK
    assert b"null" in L.frg_last_error()


@pytest.mark.parametrize("cfg", ["C1", "C2", "C3", "C5"])
def test_host_geometry_bit_exact_with_oracle(cfg):
    p = I.model_params(cfg)
    idx4 = p["N"] <= 96
    a = frg.host_tables(**p, idx4=idx4)
    b = O.Model(**p).tables(idx4=idx4)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("p", [dict(t=1.0, tp=-0.12, mu=-0.35, U=2.0, N=12, n_rad=5, n_ang=3),
                               dict(t=1.0, tp=-0.15, mu=-0.3, U=2.0, N=4, n_rad=3, n_ang=2),
                               dict(t=1.0, tp=-0.35, mu=0.0, U=2.0, N=32, n_rad=16, n_ang=16)])
def test_host_geometry_bit_exact_edge_cases(p):
    a = frg.host_tables(**p)
    b = O.Model(**p).tables()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_c4_draws_geometry_bit_exact():
    """A sample of the batched workload's seeded parameter draws."""
    flows = I.c4_flows(n_per_N=2, n_rad=4, n_ang=4)
    for p in flows:
        a = frg.host_tables(**p, idx4=False)
        b = O.Model(**p).tables(idx4=False)
        for k in a:
            assert np.array_equal(a[k], b[k]), (p, k)
