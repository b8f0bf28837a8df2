"""CPU checks of the C ABI: the library loads, exports every symbol that
include/vanse.h declares, validates arguments before touching the device,
and its host-side lattice tables agree with the paper's (matched by velocity
vector, not by index: the library has its own direction order)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vanse.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(vanse_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2208_09267_amd import vanse
    return vanse.load_library()


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["vanse_create", "vanse_set_porosity", "vanse_step", "vanse_moments",
              "vanse_destroy", "vanse_diagnostics", "vanse_init", "vanse_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2208_09267_amd import vanse
    assert sorted(vanse.EXPORTS) == _declared()


def _create(lib, lattice, dims, tau, dtype):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * 3)(*dims)
    rc = lib.vanse_create(lattice, arr, tau, dtype, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("args,needle", [
    ((7, (4, 4, 1), 0.8, 0), "lattice"),
    ((0, (4, 4, 1), 0.8, 9), "dtype"),
    ((0, (4, 4, 2), 0.8, 0), "nz"),
    ((1, (0, 4, 4), 0.8, 0), "dim"),
    ((1, (4, -1, 4), 0.8, 0), "dim"),
    ((1, (4, 4, 4), 0.5, 0), "tau"),
    ((1, (4, 4, 4), float("nan"), 0), "tau"),
    ((1, (4, 4, 4), 0.3, 1), "tau"),
    ((1, (1 << 11, 1 << 11, 1 << 10), 0.8, 0), "2^31"),
])
def test_create_rejects_bad_arguments(lib, args, needle):
    rc, h = _create(lib, *args)
    assert rc == -1 and not h.value
    assert needle in lib.vanse_last_error(None).decode()


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.vanse_step(None, 1) == -1
    assert lib.vanse_moments(None, None, None, None) == -1
    assert lib.vanse_set_porosity(None, 0.5, None, 0.0, 0) == -1
    assert lib.vanse_destroy(None) == 0
    assert lib.vanse_copy_probe(None, None, 16, None) == -1
    assert lib.vanse_set_fused(None, 2, 8) == -1
    assert lib.vanse_autotune(None, 2, None, None, None, None, None, None) == -1
    assert lib.vanse_batch_two_step_layout(None, 0, None, None) == -1


@pytest.mark.parametrize("name,lat_lib,lat_or", [("D2Q9", 0, oracle.D2Q9),
                                                 ("D3Q19", 1, oracle.D3Q19)])
def test_library_lattice_matches_oracle_by_velocity(name, lat_lib, lat_or):
    from paper_2208_09267_amd import vanse
    d, xi, w = vanse.lattice_info(lat_lib)
    d_o, c_o, w_o = oracle.lattice(lat_or)
    assert d == d_o and len(xi) == len(c_o)
    lut = {tuple(int(v) for v in c): wi for c, wi in zip(c_o, w_o)}
    for c, wi in zip(xi, w):
        assert lut[tuple(c)] == wi
    # the AA pattern relies on opp(i) = i +- H with H = (Q-1)/2
    H = (len(xi) - 1) // 2
    for i in range(1, H + 1):
        assert np.array_equal(-np.array(xi[i]), np.array(xi[i + H]))


def test_library_d3q27_matches_paper_table2():
    from paper_2208_09267_amd import vanse
    d, xi, w = vanse.lattice_info(vanse.D3Q27)
    d_o, c_o, w_o = oracle.lattice(oracle.D3Q27)
    lut = {tuple(int(v) for v in c): wi for c, wi in zip(c_o, w_o)}
    assert d == 3 and len(xi) == 27
    for c, wi in zip(xi, w):
        assert lut[tuple(c)] == wi
    for i in range(1, 14):
        assert np.array_equal(-np.array(xi[i]), np.array(xi[i + 13]))


def test_noalloc_binding_checks_buffer_sizes():
    """The C entry point takes plain device pointers; the binding checks the
    tensors' sizes before any device call (host-only: these raise on the CPU)."""
    import torch
    from paper_2208_09267_amd import vanse
    dims = (4, 3, 2)
    n = 24
    f = torch.zeros(19 * n, dtype=torch.float64)
    phi = torch.zeros(n, dtype=torch.float64)
    out = torch.zeros(7, dtype=torch.float64)
    cases = [(torch.zeros(19 * n - 1, dtype=torch.float64), phi, None, out, "f must have"),
             (f, torch.zeros(n + 1, dtype=torch.float64), None, out, "phi must have"),
             (f, phi, torch.zeros(2 * n, dtype=torch.float64), out, "force must have"),
             (f, phi, None, torch.zeros(6, dtype=torch.float64), "out must hold")]
    for ff, pp, force, oo, needle in cases:
        with pytest.raises(ValueError, match=needle):
            vanse.diagnostics_noalloc("D3Q19", dims, ff, pp, force=force, out=oo)
