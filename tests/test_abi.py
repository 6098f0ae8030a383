"""CPU checks of the C ABI: the built library loads, exports every function the
header declares, and its host-only validator returns the documented codes."""
import ctypes

import pytest
import torch

import paper_1702_04250_amd as pkg
from paper_1702_04250_amd import binding


@pytest.fixture(scope="module")
def lib():
    if not binding.LIB_PATH.exists():
        from paper_1702_04250_amd import build

        build.build()
    return pkg.load()


def test_exports_every_declared_function(lib):
    names = pkg.declared_functions()
    assert len(names) >= 15
    for n in ["pppm_validate", "pppm_plan_create", "pppm_plan_destroy", "pppm_particle_map", "pppm_make_rho",
              "pppm_poisson", "pppm_fieldforce", "pppm_compute", "pppm_energy_backward", "pppm_sync",
              "pppm_status_string", "pppm_last_error"]:
        assert n in names
    for n in names:
        assert hasattr(lib, n), n


def good(**kw):
    base = dict(box_lo=(0, 0, 0), box_len=(20.0, 21.0, 22.0), mesh=(16, 18, 20), order=5, g_ewald=0.3,
                coulomb_c=1.0, diff="ad", prec="mixed", io_dtype=torch.float32, max_particles=100)
    base.update(kw)
    return binding.make_params(**base)


def test_struct_layout_matches_c():
    # double[3] x2, int32[3], int32, double x2, 3 enums, int64, uint32 -> 112 bytes with padding
    assert ctypes.sizeof(binding.Params) == 112
    assert binding.Params.max_particles.offset == 96


@pytest.mark.parametrize("kw,code", [
    ({}, 0),
    ({"order": 1}, -2), ({"order": 8}, -2),
    ({"mesh": (4, 16, 16)}, -3),          # K < P
    ({"mesh": (1, 16, 16), "order": 2}, -3),
    ({"mesh": (4096, 16, 16)}, -3),
    ({"mesh": (2048, 2048, 2048)}, -3),  # more than 2^30 points
    ({"box_len": (0.0, 1.0, 1.0)}, -1), ({"box_len": (-1.0, 1.0, 1.0)}, -1),
    ({"box_len": (float("nan"), 1.0, 1.0)}, -1), ({"box_lo": (float("inf"), 0, 0)}, -1),
    ({"g_ewald": 0.0}, -1), ({"g_ewald": -0.3}, -1), ({"coulomb_c": 0.0}, -1),
    ({"diff": 7}, -1), ({"prec": 5}, -4), ({"io_dtype": 9}, -4),
    ({"max_particles": -1}, -1), ({"max_particles": 2 ** 31}, -1),
    ({"order": 2, "mesh": (2, 2, 2)}, 0), ({"order": 7, "mesh": (7, 9, 2048)}, 0),
])
def test_validate_codes(lib, kw, code):
    st = binding.validate(good(**kw))
    assert st == code, binding.last_error()
    if code:
        assert binding.last_error()


def test_validate_null_and_status_strings(lib):
    assert lib.pppm_validate(None) == -1
    for code, name in binding.STATUS.items():
        assert lib.pppm_status_string(code).decode().startswith(name)
    assert lib.pppm_status_string(12345) == b"unknown pppm_status"


def test_plan_calls_reject_null_plan(lib):
    assert lib.pppm_particle_map(None, 0, None, None) == -1
    assert lib.pppm_make_rho(None, None) == -1
    assert lib.pppm_sync(None) == -1
    assert lib.pppm_plan_destroy(None) == 0
    out = ctypes.c_void_p()
    assert lib.pppm_plan_create(None, None, ctypes.byref(out)) == -1
    bad = good(order=9)
    assert lib.pppm_plan_create(ctypes.byref(bad), None, ctypes.byref(out)) == -2
    assert not out.value


def test_binding_refuses_cpu_tensors_without_gpu(lib):
    if torch.cuda.is_available():
        pytest.skip("has a GPU")
    with pytest.raises(RuntimeError):
        pkg.Plan((0, 0, 0), (10, 10, 10), (8, 8, 8), 5, 0.3, max_particles=10)


@pytest.mark.parametrize("flags,code", [
    (binding.FLAG_WEIGHT_TABLE, 0),                       # default table size
    (binding.FLAG_WEIGHT_TABLE | (500 << 8), 0),
    (binding.FLAG_WEIGHT_TABLE | (65535 << 8), 0),
    (binding.FLAG_WEIGHT_TABLE | (15 << 8), -1),          # too small
    (500 << 8, -1),                                       # size without the flag
    (1 << 30, -1),                                        # unknown bit
])
def test_validate_weight_table_flags(lib, flags, code):
    p = good()
    p.flags = flags
    assert binding.validate(p) == code, binding.last_error()


def test_make_params_weight_table():
    p = good(weight_table=500)
    assert p.flags == binding.FLAG_WEIGHT_TABLE | (500 << 8)
    assert good().flags == 0


@pytest.mark.parametrize("diff,code", [("ad", 0), ("ik", -1)])
def test_validate_self_force_flag(lib, diff, code):
    # the self-force correction is defined for ad only
    p = good(diff=diff, self_force=True)
    assert p.flags == binding.FLAG_AD_SELF_FORCE
    assert binding.validate(p) == code, binding.last_error()
