"""The C-ABI library builds, loads and exports every function of include/*.h."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                             text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def libpath():
    from paper_1605_04718_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["init_problem", "destroy_problem", "forward_solve_batch",
                     "log_likelihood_batch", "mcmc_step_batch"]:
        assert required in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_binding_covers_every_symbol_and_loads(libpath):
    from paper_1605_04718_amd import _lib
    L = _lib.lib()
    for n in declared_functions():
        assert n in _lib.SYMBOLS, n
        assert hasattr(L, n)
    # error strings work without a device
    assert L.rd_status_string(-1) == b"invalid argument"


def test_null_arguments_are_rejected_without_a_device(libpath):
    from paper_1605_04718_amd import _lib
    L = _lib.lib()
    assert L.init_problem(None, None) == _lib.RD_EINVAL
    assert b"required" in L.rd_last_error()
    assert L.forward_solve_batch(None, 1, None, None, None, None, None, None, None) == _lib.RD_EINVAL
    assert L.destroy_problem(None) == _lib.RD_OK


def test_growth1d_null_arguments_are_rejected_without_a_device(libpath):
    from paper_1605_04718_amd import _lib
    L = _lib.lib()
    assert L.g1d_init(None, None) == _lib.RD_EINVAL
    assert L.g1d_forward_batch(None, 1, None, None, None, None, None) == _lib.RD_EINVAL
    assert L.g1d_log_likelihood_batch(None, 1, None, None, None, None) == _lib.RD_EINVAL
    assert L.g1d_mcmc_step_batch(None, None, 1, None) == _lib.RD_EINVAL
    assert b"NULL" in L.rd_last_error()
    assert L.g1d_destroy(None) == _lib.RD_OK


def test_growth1d_descriptor_is_validated_before_any_device_call(libpath):
    """n outside [2, 128] and a missing initial field are call errors that
    need no device."""
    import ctypes
    import numpy as np
    from paper_1605_04718_amd import _lib
    L = _lib.lib()
    u = np.ones(200)
    d = _lib.G1dDesc()
    d.n, d.n_steps, d.tau, d.rho_T, d.max_batch = 129, 10, 1e-4, 1.8, 4
    d.theta[:] = [0.1, 0.9, 1000.0, 10.0]
    d.u0 = d.v0 = u.ctypes.data_as(_lib.c_dp)
    h = ctypes.c_void_p()
    assert L.g1d_init(ctypes.byref(d), ctypes.byref(h)) == _lib.RD_EINVAL
    assert b"n = 129" in L.rd_last_error()
    d.n = 100
    d.v0 = None
    assert L.g1d_init(ctypes.byref(d), ctypes.byref(h)) == _lib.RD_EINVAL
    assert b"u0 and v0" in L.rd_last_error()
