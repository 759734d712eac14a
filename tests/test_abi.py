"""The C ABI: every entry point declared in include/nepmi.h is exported by the
built library and bound by the Python layer; host-only calls (no GPU work)
agree with the FP64 oracle's independent implementation."""
import ctypes as C
import re
from pathlib import Path

import pytest

from paper_2607_06969_amd import workloads as W

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "nepmi.h"


def declared():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nepmi_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2607_06969_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.skip("libnepmi.so not built")
    return _lib


def test_every_declared_symbol_is_exported_and_bound(lib):
    names = declared()
    assert len(names) >= 20
    L = C.CDLL(str(lib.LIB_PATH))
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in lib.SIGNATURES}
    assert bound == set(names), (set(names) - bound, bound - set(names))


@pytest.mark.parametrize("hpf", [W.hp_small_single, W.hp_gst, W.hp_table2])
def test_sizes_agree_with_oracle(lib, oracle_lib, hpf):
    hp = hpf()
    assert lib.param_count(hp) == oracle_lib.param_count(hp) == hp.n_params()
    assert lib.descriptor_dim(hp) == oracle_lib.descriptor_dim(hp) == hp.dim
    assert lib.supported(hp)


def test_table2_has_7899_parameters(lib):
    assert lib.param_count(W.hp_table2()) == 7899


def test_invalid_and_unsupported_hparams(lib):
    from paper_2607_06969_amd._lib import HParams, NepmiError, load
    bad = W.hp_gst()
    bad.rc_angular = 7.0  # larger than the radial cutoff
    with pytest.raises(NepmiError) as e:
        lib.param_count(bad)
    assert e.value.code == lib.INVALID_ARG
    odd = W.hp_gst()
    odd.n_hidden = 17  # valid model, no compiled kernels
    assert lib.param_count(odd) == odd.n_params()
    assert not lib.supported(odd)
    h = C.c_void_p()
    assert load().nepmi_model_create(C.byref(HParams.from_any(odd)), C.byref(h)) == lib.UNSUPPORTED
