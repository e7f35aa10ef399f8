"""C-ABI checks that need no GPU: the library loads, exports every function that
include/melt.h declares, and rejects bad arguments before touching a device."""
import ctypes
import re
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    text = (ROOT / "include" / "melt.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n.startswith(("melt_", "stft_"))))


@pytest.fixture(scope="module")
def lib():
    import paper_2606_01009_amd as m
    if not m.library_path().exists():
        pytest.skip("libmelt.so not built")
    return m


def test_header_declares_the_boundary():
    d = _declared()
    for name in ("melt_plan_create", "melt_forward", "melt_backward", "stft_mel_forward", "melt_stream_push"):
        assert name in d


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", str(lib.library_path())], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    assert set(_declared()) == set(lib.exported_symbols())


def test_host_only_entry_points(lib):
    lib.load_library()
    assert lib.melt_num_frames(16000, 400, 160) == 98
    assert lib.melt_num_frames(399, 400, 160) == 0
    assert lib.melt_num_frames(10, 0, 160) == -1
    c = lib.melt_config_default()
    assert (c.n_fft, c.hop, c.n_mels, c.sample_rate, c.fmax) == (400, 160, 80, 16000.0, 8000.0)
    assert lib.melt_status_string(lib.MELT_E_SHAPE) == "MELT_E_SHAPE"


@pytest.mark.parametrize("field,value", [("n_fft", 1), ("n_fft", 5000), ("hop", 0), ("n_mels", 0), ("n_mels", 600),
                                         ("fmax", 9000.0), ("fmin", -1.0), ("log_eps", 0.0), ("log_eps", 1e-39), ("precision", 9),
                                         ("output", 7), ("sample_rate", 0.0)])
def test_invalid_configs_rejected(lib, field, value):
    c = lib.melt_config_default()
    setattr(c, field, value)
    h = ctypes.c_void_p()
    st = lib.load_library().melt_plan_create(ctypes.byref(c), 0, ctypes.byref(h))
    assert st == lib.MELT_E_INVALID_ARG
    assert h.value is None


@pytest.mark.parametrize("n_fft,hop", [(400, 401), (256, 270), (16, 65536)])
def test_hop_beyond_frame_is_unsupported(lib, n_fft, hop):
    """Frames that skip samples (hop > n_fft) are rejected with MELT_E_UNSUPPORTED before
    any device call; hop == n_fft (adjacent frames) is a valid configuration."""
    c = lib.melt_config_default()
    c.n_fft, c.hop = n_fft, hop
    h = ctypes.c_void_p()
    assert lib.load_library().melt_plan_create(ctypes.byref(c), 0, ctypes.byref(h)) == lib.MELT_E_UNSUPPORTED
    assert h.value is None
    assert "hop > n_fft" in lib.melt_last_error()


def test_null_arguments_rejected(lib):
    L = lib.load_library()
    assert L.melt_plan_create(None, 0, None) == lib.MELT_E_INVALID_ARG
    assert L.melt_forward(None, None, None, 0, 0, None, None) == lib.MELT_E_INVALID_ARG
    assert L.melt_plan_destroy(None) == lib.MELT_OK
    assert L.melt_variant_count(None) == 0
    assert L.melt_variant_name(None, 0) == b"none"
    assert L.melt_set_variant(None, 0, 0) == lib.MELT_E_INVALID_ARG
