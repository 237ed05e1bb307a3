"""The C-ABI library loads and exports every symbol include/mcwind.h declares,
and its host-side argument checks work without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcwind.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcw_[A-Za-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2101_08453_amd import mcwind
    if not os.path.exists(mcwind.LIB_PATH):
        pytest.fail("libmcwind.so is not built (python -m paper_2101_08453_amd.build)")
    return mcwind.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for need in ["mcw_create", "mcw_solve", "mcw_solve_batch", "mcw_adjoint", "mcw_destroy",
                 "mcw_apply_K", "mcw_rhs", "mcw_recover", "mcw_divergence", "mcw_smooth",
                 "mcw_residual", "mcw_restrict", "mcw_prolong", "mcw_coarse_solve",
                 "mcw_get_stencil", "mcw_level_info", "mcw_status_string", "mcw_last_error"]:
        assert need in names


# Calls that run an operation of the method; each must cite the passage that
# defines it.  The rest are lifetime, error, option, tolerance and timing calls.
OPERATIONS = ["mcw_create", "mcw_solve", "mcw_solve_batch", "mcw_adjoint", "mcw_apply_K",
              "mcw_rhs", "mcw_recover", "mcw_divergence", "mcw_interp_wind", "mcw_surface_wind",
              "mcw_num_levels", "mcw_level_info", "mcw_get_stencil", "mcw_smooth",
              "mcw_residual", "mcw_restrict", "mcw_prolong", "mcw_coarse_solve", "mcw_vcycle"]


def test_every_operation_cites_its_defining_passage():
    """The comment block in front of each operation's declaration names a
    section or an equation of the paper."""
    text = open(HEADER).read()
    for name in OPERATIONS:
        m = re.search(r"(?m)^[A-Za-z_][\w \*]*\b" + name + r"\s*\(", text)  # the declaration
        assert m, name
        head = text[:m.start()].rstrip()
        if name == "mcw_level_info":  # shares the comment of mcw_num_levels
            head = head[:head.rfind("\n")].rstrip()
        assert head.endswith("*/"), f"{name} has no comment block"
        block = head[head.rfind("/*"):]
        assert re.search(r"Sec\. \d|eqs?\. \(\d\)", block), f"{name} cites no passage"


def test_library_exports_every_declared_symbol(lib):
    from paper_2101_08453_amd import mcwind
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in mcwind.SIGNATURES, f"binding lacks {name}"


def test_status_strings_and_defaults(lib):
    from paper_2101_08453_amd import mcwind
    for s, name in enumerate(mcwind.STATUS_NAMES):
        assert lib.mcw_status_string(s).decode() == name
    o = mcwind.default_options()
    assert o.precision == mcwind.FP32_REFINE and o.rtol == 1e-8
    assert (o.nu_pre, o.nu_post, o.coarsen_rule, o.use_graph) == (2, 2, 0, 1)
    # the last fields: a layout mismatch with the header would read other values here
    assert (o.krylov, o.smoother, o.stencil_fp16) == (0, 0, 0)
    assert o.merge_spacing == 0 and o.tune_cache is None


def test_create_rejects_bad_arguments_on_the_host(lib):
    from paper_2101_08453_amd import mcwind
    h = mcwind.H()
    assert lib.mcw_create(None, None, None, ctypes.byref(h)) == 1
    d = mcwind.GridDesc()
    d.nx, d.ny, d.nz = 1, 4, 4  # nx < 2
    d.X = d.Y = d.Z = ctypes.c_void_p(16)
    d.a[0] = d.a[1] = d.a[2] = 1.0
    d.gamma_faces = 1
    assert lib.mcw_create(ctypes.byref(d), None, None, ctypes.byref(h)) == 1
    d.nx = 4
    d.a[2] = 0.0  # a_3 <= 0
    assert lib.mcw_create(ctypes.byref(d), None, None, ctypes.byref(h)) == 1
    assert b"penalty" in lib.mcw_last_error(None)
    d.a[2] = 1.0
    d.gamma_faces = 63  # Gamma = every face
    assert lib.mcw_create(ctypes.byref(d), None, None, ctypes.byref(h)) == 3
    o = mcwind.default_options()
    d.gamma_faces = 1
    o.coarse_direct_max = 0
    assert lib.mcw_create(ctypes.byref(d), ctypes.byref(o), None, ctypes.byref(h)) == 1
    o = mcwind.default_options()
    o.precision = mcwind.FP64
    o.stencil_fp16 = 1  # FP16 stencils serve the FP32 V-cycle only
    assert lib.mcw_create(ctypes.byref(d), ctypes.byref(o), None, ctypes.byref(h)) == 1
    assert b"stencil_fp16" in lib.mcw_last_error(None)
    o.precision = mcwind.FP32_REFINE
    o.stencil_fp16 = 2
    assert lib.mcw_create(ctypes.byref(d), ctypes.byref(o), None, ctypes.byref(h)) == 1
    o = mcwind.default_options()
    o.merge_spacing = 2
    assert lib.mcw_create(ctypes.byref(d), ctypes.byref(o), None, ctypes.byref(h)) == 1
    assert b"merge_spacing" in lib.mcw_last_error(None)
    assert not h.value


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.mcw_solve(None, None, None, None, None) == 1
    assert lib.mcw_num_levels(None) == 0
    lib.mcw_destroy(None)
