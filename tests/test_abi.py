"""C-ABI tests that need no GPU: exported symbols, validation, error codes."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_20507_amd import ammse, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ammse.h")


def _declared_functions():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ammse_status_t|int32_t|const char\*|void)\s+"
                                 r"(ammse_\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ammse.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return ammse.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert len(names) == 15
    assert set(names) == set(ammse.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_version_and_status_strings(L):
    assert L.ammse_version() == 2
    for code in range(0, 9):
        s = L.ammse_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0


def test_struct_layout_matches_header():
    assert ctypes.sizeof(ammse.AmmseInstance) == 56
    assert ammse.AmmseInstance.h_off.offset == 24
    assert ctypes.sizeof(ammse.AmmseOptions) == 80
    assert ammse.AmmseOptions.algorithm.offset == 40
    assert ammse.AmmseOptions.tile.offset == 44
    assert ammse.AmmseOptions.step_rule.offset == 48
    assert ammse.AmmseOptions.eps1.offset == 56


def test_default_options_match_paper(L):
    o = ammse.AmmseOptions()
    L.ammse_default_options(ctypes.byref(o))
    assert (o.precision, o.max_iters, o.T_c, o.warm_start, o.extrapolate) == (1, 100, 3, 1, 1)
    assert o.eps1 == pytest.approx(0.1) and o.eps2 == 0.0 and o.force_switch_iter == -1
    assert o.refine_iters == 10 and o.algorithm == ammse.ALGO_AMMMSE and o.tile == 0
    assert o.step_rule == ammse.STEP_BOUND and o.gamma_c == 0.0 and o.rearm_at_switch == 1


def test_validate_reports_buffer_lengths(L):
    b = synth.hexcell_batch(B=5)
    table, cu = ammse.make_table(b)
    h, v, u, s = ammse.validate(table, cu)
    assert h == b.H.size and v == b.V0.size and u == b.sigma2.size and s == b.P.size


def _one(**kw):
    b = synth.rayleigh_batch(1, 2, M=8, U=3, N=2, d=2, P=1.0)
    table, cu = ammse.make_table(b)
    for k, val in kw.items():
        setattr(table[0], k, val)
    return table, cu


@pytest.mark.parametrize("field,value,code", [
    ("d", 3, 2), ("N", 0, 2), ("M", 0, 2), ("C", 0, 2), ("U", 4, 2), ("h_off", -1, 2),
    ("N", 5, 6), ("C", 17, 6), ("cell_off", -2, 2),
])
def test_validate_rejects_bad_shapes(L, field, value, code):
    table, cu = _one(**{field: value})
    if field == "N" and value == 5:
        table[0].d = 1
    with pytest.raises(ammse.AmmseError) as e:
        ammse.validate(table, cu)
    assert e.value.code == code


def test_validate_rejects_overlapping_precoders(L):
    table, cu = _one()
    table[1].v_off = table[0].v_off + 1
    with pytest.raises(ammse.AmmseError) as e:
        ammse.validate(table, cu)
    assert e.value.code == 2


@pytest.mark.parametrize("opt", [
    dict(precision=7), dict(max_iters=-1), dict(T_c=-1), dict(lanczos_steps=65),
    dict(force_switch_iter=0), dict(eps1=-0.1), dict(T_c=0), dict(eps2=float("nan")),
    dict(path=2), dict(refine_iters=-1), dict(precision=3),
    dict(tile=4), dict(tile=-1), dict(step_rule=2), dict(step_rule=-1), dict(algorithm=4),
])
def test_validate_rejects_bad_options(L, opt):
    table, cu = _one()
    with pytest.raises(ammse.AmmseError) as e:
        ammse.validate(table, cu, ammse.Options(**opt))
    assert e.value.code == 3


@pytest.mark.parametrize("algo", [ammse.ALGO_WMMSE, ammse.ALGO_MMMSE, ammse.ALGO_BCGD])
def test_other_algorithms_in_bfloat16_are_unsupported(L, algo):
    table, cu = _one()
    with pytest.raises(ammse.AmmseError) as e:
        ammse.validate(table, cu, ammse.Options(algorithm=algo, precision=ammse.PREC_BF16))
    assert e.value.code == 6


def test_empty_batch_is_valid_but_cannot_be_planned(L):
    assert ammse.validate([], np.zeros(0, np.int32)) == (0, 0, 0, 0)


def test_plan_create_validates_before_touching_the_device(L):
    table, cu = _one(d=3)
    h = ctypes.c_void_p()
    opt = ammse.Options().to_c()
    code = L.ammse_plan_create(ctypes.byref(h), 0, table,
                               cu.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), 2,
                               ctypes.byref(opt))
    assert code == 2 and not h.value
    assert L.ammse_plan_create(None, 0, table, None, 2, ctypes.byref(opt)) == 1


def test_null_arguments(L):
    assert L.ammse_plan_workspace_size(None, None) == 1
    assert L.ammse_plan_destroy(None) == 0
    assert L.ammse_plan_info(None, None, None) == 1
    assert L.ammse_solve(None, *([None] * 12), 0, None) == 1
    assert L.ammse_wsr(None, *([None] * 6), 0, None) == 1
