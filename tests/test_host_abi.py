"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function the header declares, descriptor validation refuses
bad input with SCP_EINVAL before any device work, and the serving footprint
estimate behaves."""
import copy
import ctypes as C
import os
import re

import pytest

import scp_inputs as si

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scprop.h")

_libmod = pytest.importorskip("paper_2406_18155_amd._lib")
if not os.path.exists(_libmod.LIB_PATH):
    pytest.skip("libscprop.so is not built (run __graft_entry__.build())", allow_module_level=True)

from paper_2406_18155_amd._lib import EXPORTS, SCP_EINVAL, SCP_OK, lib  # noqa: E402
from paper_2406_18155_amd.api import marshal  # noqa: E402


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(scp_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_compute_and_serving_calls():
    names = declared_functions()
    for n in ("scp_build_system", "scp_propagate", "scp_propagate_adjoint", "scp_fidelity",
              "scp_server_step", "scp_last_error"):
        assert n in names


def test_library_exports_every_declared_function():
    L = C.CDLL(_libmod.LIB_PATH)
    names = declared_functions()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # the ctypes table declares exactly the header's functions
    assert sorted(EXPORTS) == names


def _build(desc):
    sd, keep = marshal(desc)
    h = C.c_void_p()
    st = lib().scp_build_system(C.byref(sd), None, C.byref(h))
    return st, lib().scp_last_error().decode()


def _bad_cases():
    base = si.config1()
    cases = []
    d = copy.deepcopy(base)
    d["modes"][1]["trunc"] = 9
    cases.append(("truncation above the maximum", d, "trunc out of range"))
    d = copy.deepcopy(base)
    d["couplings"][0]["op_i"] = "phi"
    cases.append(("transmon phase coupling", d, "phase operator"))
    d = copy.deepcopy(base)
    d["drives"][0]["op"] = "phi"
    cases.append(("transmon phase drive", d, "phase operator"))
    d = copy.deepcopy(base)
    d["drives"][0]["params"] = [0.1, 0.2]
    cases.append(("two parameters for a Gaussian", d, "one parameter"))
    d = copy.deepcopy(base)
    d["drives"][0]["sigma"] = 0.0
    cases.append(("zero sigma", d, "sigma"))
    d = copy.deepcopy(base)
    d["drives"][0]["params"] = [float("nan")]
    cases.append(("NaN amplitude", d, "non-finite"))
    d = copy.deepcopy(base)
    d["couplings"][0]["j"] = d["couplings"][0]["i"]
    cases.append(("self coupling", d, "coupling modes"))
    d = copy.deepcopy(base)
    d["n_steps"] = 0
    cases.append(("zero steps", d, "n_steps"))
    d = copy.deepcopy(base)
    d["T"] = -1.0
    cases.append(("negative T", d, "T must be"))
    d = copy.deepcopy(base)
    d["modes"][0]["basis_dim"] = 20
    cases.append(("even charge basis", d, "basis_dim"))
    d = copy.deepcopy(si.config2())
    d["modes"][0]["EL"] = 0.0
    cases.append(("fluxonium without inductance", d, "EL"))
    return cases


@pytest.mark.parametrize("name,desc,msg", _bad_cases(), ids=[c[0] for c in _bad_cases()])
def test_invalid_descriptions_are_refused_before_device_work(name, desc, msg):
    st, err = _build(desc)
    assert st == SCP_EINVAL, (st, err)
    assert msg in err, err


def test_null_arguments_are_refused():
    h = C.c_void_p()
    assert lib().scp_build_system(None, None, C.byref(h)) == SCP_EINVAL
    sd, keep = marshal(si.config1())
    assert lib().scp_build_system(C.byref(sd), None, None) == SCP_EINVAL
    n = C.c_size_t()
    assert lib().scp_request_bytes(None, 4, 0, C.byref(n)) == SCP_EINVAL
    assert lib().scp_request_bytes(C.byref(sd), 0, 0, C.byref(n)) == SCP_EINVAL
    srv = C.c_void_p()
    assert lib().scp_server_create(0, 4, 0.0, None, C.byref(srv)) == SCP_EINVAL
    assert lib().scp_server_create(1 << 30, 0, 0.0, None, C.byref(srv)) == SCP_EINVAL
    rf = C.c_int32()
    assert lib().scp_system_frame(None, C.byref(rf)) == SCP_EINVAL
    assert lib().scp_system_set_frame(None, 0) == SCP_EINVAL
    assert lib().scp_trotter_workspace_size(None, 1, C.byref(n)) == SCP_EINVAL
    assert lib().scp_propagate_trotter(None, 1, 1, None, None, None, None) == SCP_EINVAL
    assert lib().scp_propagate_adjoint(None, None, None, None, None, None, None) == SCP_EINVAL
    assert lib().scp_fidelity_states(None, 4, 1, 0, 1, None, None, None, None, None,
                                     None) == SCP_EINVAL


def test_request_footprint_grows_with_columns_steps_and_gradient():
    def nbytes(desc, cols, grad):
        sd, keep = marshal(desc)
        n = C.c_size_t()
        assert lib().scp_request_bytes(C.byref(sd), cols, grad, C.byref(n)) == SCP_OK
        return n.value

    q = si.serving_request(0)
    S = len(q["columns"])
    D = q["modes"][0]["trunc"] ** len(q["modes"])
    fwd, grad = nbytes(q, S, 0), nbytes(q, S, 1)
    assert fwd >= 4 * S * D * 8          # psi, hi, lo, costate in complex64
    assert grad > fwd
    assert nbytes(q, 2 * S, 1) > grad
    longer = copy.deepcopy(q)
    longer["n_steps"] *= 4
    assert nbytes(longer, S, 1) > grad


def test_padded_indices_map_product_states_to_the_uniform_index_space():
    # modes truncated to (3, 2, 4) run at d = 4: level a_m of mode m sits at
    # stride 4^(2 - m); brute force over every product state
    from paper_2406_18155_amd import padded_indices
    exp = [(a * 4 + b) * 4 + c for a in range(3) for b in range(2) for c in range(4)]
    assert padded_indices([3, 2, 4], range(24)) == exp
    assert padded_indices([4, 4], range(16)) == list(range(16))
    with pytest.raises(ValueError):
        padded_indices([2, 3], [6])


def test_header_compiles_as_c11():
    # include/scprop.h is a C header: it compiles as C11 with every warning
    # an error (the C ABI must not need a C++ compiler)
    import shutil
    import subprocess
    import tempfile
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "h.c")
        with open(src, "w") as f:
            f.write('#include "scprop.h"\nint main(void) { return SCP_OK; }\n')
        subprocess.check_call([gcc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic",
                               "-fsyntax-only", "-I", os.path.join(root, "include"), src])
