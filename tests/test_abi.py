"""CPU-side checks of the C ABI: the library loads, exports every symbol include/vbc.h
declares, and its host-only validation (vbc_workspace_size) rejects bad parameter sets
with the documented status codes.  No GPU call is made here."""
import ctypes as C
import os
import re

import pytest

from paper_2609_07842_amd import vbc
from paper_2609_07842_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "vbc.h")).read()
    return sorted(set(re.findall(r"^(?:vbc_status|const char \*)\s*(vbc_\w+)\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    L = vbc.lib()
    declared = _declared_symbols()
    assert len(declared) >= 13
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(vbc.EXPORTS)


def test_workspace_size_grows_with_n():
    p = W.vbc_params(E_a=5.0, f=2.0)
    a = vbc.workspace_size([vbc.replica(1000, W.box_length(1000, 0.3), p)])
    b = vbc.workspace_size([vbc.replica(100000, W.box_length(100000, 0.3), p)])
    assert 0 < a < b


@pytest.mark.parametrize("bad,status", [
    (dict(E_r=-1.0), vbc.VBC_ERR_ARG),
    (dict(r_a=0.9), vbc.VBC_ERR_ARG),        # r_a < r_r
    (dict(r_h=1.0, r_l=1.5), vbc.VBC_ERR_ARG),
    (dict(E_a=float("nan")), vbc.VBC_ERR_ARG),
])
def test_invalid_parameters_rejected(bad, status):
    p = W.vbc_params(**bad) if "E_a" not in bad else dict(W.vbc_params(), **bad)
    with pytest.raises(vbc.VBCError) as ei:
        vbc.workspace_size([vbc.replica(100, 20.0, p)])
    assert ei.value.status == status


def test_box_too_small_rejected():
    with pytest.raises(vbc.VBCError) as ei:
        vbc.workspace_size([vbc.replica(50, 4.7, W.vbc_params())])  # 2 * 2.4 > 4.7
    assert ei.value.status == vbc.VBC_ERR_BOX
    # just large enough: three cells per axis
    assert vbc.workspace_size([vbc.replica(50, 7.3, W.vbc_params())]) > 0


def test_asymmetric_pair_table_rejected():
    a = W.vbc_params(E_a=1.0)
    b = W.vbc_params(E_a=2.0)
    with pytest.raises(vbc.VBCError) as ei:
        vbc.workspace_size([vbc.replica(100, 20.0, [a, a, b, a])])
    assert ei.value.status == vbc.VBC_ERR_ARG


def test_option_validation():
    p = W.vbc_params()
    r = vbc.replica(100, 20.0, p)
    for kw in (dict(brick=7), dict(block=100), dict(k_max=70000)):
        with pytest.raises(vbc.VBCError):
            vbc.workspace_size([r], **kw)
    with pytest.raises(vbc.VBCError):
        vbc.workspace_size([vbc.replica(100, 20.0, [p] * 25)])  # 5 types > 4


def test_chain_length_must_divide_n():
    with pytest.raises(vbc.VBCError):
        vbc.workspace_size([vbc.replica(101, 20.0, W.vbc_params(), chain_len=10, k_bond=100.0)])


def test_empty_inputs_rejected():
    # a replica without particles, and a call without replicas, are argument errors
    with pytest.raises(vbc.VBCError) as ei:
        vbc.workspace_size([vbc.replica(0, 20.0, W.vbc_params())])
    assert ei.value.status == vbc.VBC_ERR_ARG
    with pytest.raises(vbc.VBCError) as ei:
        vbc.workspace_size([])
    assert ei.value.status == vbc.VBC_ERR_ARG
