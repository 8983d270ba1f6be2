"""CPU checks of the C ABI: the library loads and exports every declared symbol.

No compute call is made here (there is no GPU in the build container).
"""
import ctypes
import os
import re

import pytest

from paper_2207_05612_amd import mps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mps_dmrg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_abi():
    names = declared_functions()
    for required in ("mps_create", "mps_destroy", "apply_layer_dmrg", "fidelity", "sample"):
        assert required in names
    assert set(names) == set(mps.EXPORTS)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(mps.LIB_PATH):
        pytest.fail("libmpsdmrg.so is not built; run `python -m paper_2207_05612_amd.build`")
    lib = ctypes.CDLL(mps.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_fails_loudly_without_library(tmp_path):
    saved = mps._lib
    mps._lib = None
    try:
        with pytest.raises(ImportError):
            mps.load_library(str(tmp_path / "missing.so"))
    finally:
        mps._lib = saved


def test_gate_record_layout():
    # mps_gate = {int32 q0, int32 q1, double m[32]} without padding: 264 bytes
    from paper_2207_05612_amd import circuits
    import numpy as np
    assert circuits.GATE_DTYPE.itemsize == 264
    rec = circuits.pack_layer([(3, -1, circuits.SQRT_X), (0, 5, circuits.fsim(0.3, 0.2))])
    assert rec[0]["q1"] == -1 and rec[1]["q0"] == 0 and rec[1]["q1"] == 5
    m = rec[1]["m"][0::2] + 1j * rec[1]["m"][1::2]
    assert np.allclose(m.reshape(4, 4), circuits.fsim(0.3, 0.2))
