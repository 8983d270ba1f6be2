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
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\b\s*\*?\s*([a-z_0-9]+)\s*\(", text, flags=re.M)))


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


def _prototype(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    m = re.search(r"\b%s\s*\((.*?)\)\s*;" % name, text, flags=re.S)
    assert m, name
    return [" ".join(a.split()) for a in m.group(1).split(",")]


def test_create_takes_allocator_callbacks():
    args = _prototype("mps_create")
    assert args == ["int n_sites", "const uint8_t* init_bits", "int max_chi", "int precision",
                    "void* hip_stream", "const mps_allocator* alloc", "mps_state** out"]
    # struct mps_allocator: alloc, free, user -- three pointers, as the binding declares it
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\}\s*mps_allocator;", text, flags=re.S).group(1)
    fields = [f.strip() for f in body.split(";") if f.strip()]
    assert fields[0].startswith("void* (*alloc)(size_t bytes, void* stream, void* user")
    assert fields[1].startswith("void (*free)(void* ptr, void* stream, void* user")
    assert fields[2] == "void* user"
    assert ctypes.sizeof(mps.MpsAllocator) == 3 * ctypes.sizeof(ctypes.c_void_p)
    assert [f[0] for f in mps.MpsAllocator._fields_] == ["alloc", "free", "user"]


def test_precision_values_match_the_header():
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = dict((k, int(v)) for k, v in re.findall(r"\b(MPS_(?:FP64|FP32|BF16X2|BF16X3))\s*=\s*(\d+)", text))
    assert vals == {"MPS_FP64": mps.MPS_FP64, "MPS_FP32": mps.MPS_FP32, "MPS_BF16X2": mps.MPS_BF16X2,
                    "MPS_BF16X3": mps.MPS_BF16X3}
