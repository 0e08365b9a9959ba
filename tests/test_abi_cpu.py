"""CPU-only checks of the C ABI: the built library loads, exports every symbol
include/hevmc.h declares, and rejects invalid arguments without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1312_1282_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hevmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hevmc_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_binding_exports():
    assert _declared() == sorted(abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = abi.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_status_codes_match_the_header():
    """Every hevmc_status the header defines has the binding's name and value."""
    with open(os.path.join(ROOT, "include", "hevmc.h")) as fh:
        text = fh.read()
    body = text[text.index("typedef enum {"):text.index("} hevmc_status;")]
    codes = {int(v): k for k, v in re.findall(r"(HEVMC_[A-Z]+)\s*=\s*(-?\d+)", body)}
    assert codes == abi.STATUS


def test_parameter_struct_layouts():
    assert C.sizeof(abi.Params) == 72
    assert C.sizeof(abi.WalkerAcc) == 160
    assert C.sizeof(abi.Plan) == 40


@pytest.mark.parametrize("bad", [
    dict(n=1), dict(n_walkers=0), dict(precision=7), dict(order=3), dict(density=0.0),
    dict(density=float("nan")), dict(b=-1.0), dict(hbar2_over_m=0.0), dict(step_sigma=0.0),
    dict(threads=96), dict(variant=3),
])
def test_invalid_parameters_rejected(bad):
    kw = dict(n=108, n_walkers=4)
    kw.update(bad)
    p = abi.make_params(**kw)
    with pytest.raises(abi.HevmcError) as ei:
        abi.box(p)
    assert ei.value.code == -1


def test_box_side():
    p = abi.make_params(108, 1, density=0.02186)
    import oracle as O
    assert abi.box(p) == O.box_side(108, 0.02186)
    p32 = abi.make_params(108, 1, density=0.02186, precision=abi.FP32)
    assert abi.box(p32) == O.box_side(108, 0.02186, fp32=True)


def test_error_string_is_set():
    with pytest.raises(abi.HevmcError, match="need at least 2 atoms"):
        abi.box(abi.make_params(1, 1))
