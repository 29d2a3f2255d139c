"""The C-ABI library loads and exports every symbol that include/tpmvs.h
declares (host-side checks, no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tpmvs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tpm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_expected_calls():
    names = _declared()
    for must in ("tpm_create", "tpm_set_central", "tpm_set_planets", "tpm_set_particles",
                 "tpm_integrate", "tpm_get_particles", "tpm_get_planets", "tpm_destroy",
                 "tpm_last_error", "tpm_hill_radius"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2011_03484_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name
    assert set(_lib.SIGNATURES) == set(_declared())


def test_hill_radius_host_helper():
    from paper_2011_03484_amd import _lib
    assert abs(_lib.hill_radius(1.0, 3e-3, 2.0) - 0.2) < 1e-15


def test_create_without_gpu_reports_device_error():
    """With no usable gfx950 device the library returns TPM_EDEVICE (it never
    falls back to the CPU)."""
    from paper_2011_03484_amd import _lib
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(_lib.TpmError) as e:
        _lib.Simulation()
    assert e.value.code == _lib.TPM_EDEVICE


def test_invalid_arguments_refused_before_device_work():
    """Argument checks come first: these calls fail with TPM_EINVAL on any
    machine, GPU or not, without touching the device."""
    from paper_2011_03484_amd import _lib
    for bad in ([1.0, 0.0], [-1.0], [float("nan")], [float("inf")]):
        with pytest.raises(_lib.TpmError) as e:
            _lib.debug_rsqrt(bad)
        assert e.value.code == _lib.TPM_EINVAL, bad
    with pytest.raises(_lib.TpmError) as e:
        _lib.Simulation(chunk_steps=(1 << 30) + 1)
    assert e.value.code == _lib.TPM_EINVAL
    with pytest.raises(_lib.TpmError) as e:
        _lib.Simulation(waves_per_simd=9)
    assert e.value.code == _lib.TPM_EINVAL
    with pytest.raises(_lib.TpmError) as e:
        _lib.Simulation(kepler_iters=65)
    assert e.value.code == _lib.TPM_EINVAL
    from paper_2011_03484_amd import workloads as W
    w = W.single_planet(n=4, seed=1)
    for kw in ({"kepler_iters": 65}, {"chunk_steps": (1 << 30) + 1}, {"block_threads": 96}):
        with pytest.raises(_lib.TpmError) as e:
            _lib.batch_integrate([w], nsteps=10, **kw)
        assert e.value.code == _lib.TPM_EINVAL, kw
