"""Host-side checks of the C ABI (no GPU): the library loads, exports every entry
point that include/hub.h declares, the ctypes structs match the header's layout,
and argument errors are reported without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hub.h")
LIB = os.path.join(ROOT, "paper_1804_07195_amd", "libhub.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hub_[a-z_A-Z]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1804_07195_amd.build_lib import build
        build()
    from paper_1804_07195_amd import binding
    return binding.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ["hub_apply_M", "hub_apply_Mdag", "hub_solve", "hub_force", "hub_force_sum", "hub_submit", "hub_poll",
              "hub_create", "hub_destroy", "hub_last_error", "hub_action", "hub_apply_normal", "hub_default_opts",
              "hub_profile_enable", "hub_profile_read", "hub_hasenbusch_heatbath", "hub_hasenbusch_force",
              "hub_md_schedule", "hub_hmc_trajectory", "hub_hmc_trajectories", "hub_solve_multishift", "hub_hasenbusch_masses"]:
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_lists_every_symbol():
    from paper_1804_07195_amd import binding
    assert sorted(binding.SYMBOLS) == declared_functions()


def test_struct_layouts_match_header():
    from paper_1804_07195_amd import binding as b
    assert ctypes.sizeof(b.HubLattice) == 32
    assert b.HubLattice.kappa_t.offset == 16
    assert ctypes.sizeof(b.HubSolveOpts) == 48
    assert b.HubSolveOpts.tol.offset == 16 and b.HubSolveOpts.use_x0.offset == 40
    assert ctypes.sizeof(b.HubSolveInfo) == 24
    assert b.HubSolveInfo.true_rel_resid.offset == 16
    assert b.HubRequest.opts.offset == 80
    assert ctypes.sizeof(b.HubKernelStat) == 40
    assert ctypes.sizeof(b.HubHmcParams) == 232
    assert b.HubHmcParams.n.offset == 28 and b.HubHmcParams.mt.offset == 32 and b.HubHmcParams.n_scale.offset == 160
    assert ctypes.sizeof(b.HubMdOp) == 152 and b.HubMdOp.coef.offset == 16
    assert ctypes.sizeof(b.HubHmcInfo) == 120
    assert b.HubHmcInfo.inner_iters.offset == 40 and b.HubHmcInfo.force_evals.offset == 48


def test_default_options(lib):
    from paper_1804_07195_amd import binding as b
    o = b.default_opts()
    assert (o.solver, o.max_iter, o.restart_m, o.inner_max_iter) == (b.HUB_CG_FP64, 20000, 10, 4000)
    assert (o.tol, o.inner_a, o.inner_floor, o.use_x0, o.check_every) == (1e-10, 5.0, 1e-5, 0, 8)


def test_argument_errors_without_a_device(lib):
    from paper_1804_07195_amd import binding as b
    lat = b.lattice(3, 3, 8, 0.5)
    # NULL context and NULL buffers are rejected before any HIP call
    assert lib.hub_apply_M(None, ctypes.byref(lat), None, None, None, 1, None) == b.HUB_ERR_ARG
    assert b"NULL" in lib.hub_last_error()
    assert lib.hub_create(None, 0, 0) == b.HUB_ERR_ARG
    info = b.HubSolveInfo()
    assert lib.hub_solve(None, ctypes.byref(lat), None, None, 1, None, None, None, ctypes.byref(info), None) \
        == b.HUB_ERR_ARG
    done = ctypes.c_int32()
    assert lib.hub_poll(None, ctypes.c_uint64(1), ctypes.byref(done), None) == b.HUB_ERR_ARG
    hinfo = b.HubHmcInfo()
    p = b.hmc_params(0.5, 4)
    assert lib.hub_hmc_trajectory(None, ctypes.byref(lat), None, None, None, 0.5, ctypes.byref(p), None,
                                  ctypes.byref(hinfo), None) == b.HUB_ERR_ARG
    assert lib.hub_hasenbusch_heatbath(None, ctypes.byref(lat), None, None, 0, None, None, None, None,
                                       None) == b.HUB_ERR_ARG


def test_hasenbusch_masses_host_helper(lib):
    from oracle.multishift import hasenbusch_masses
    from paper_1804_07195_amd import binding as b
    for n in (1, 2, 5):
        got = b.hub_hasenbusch_masses(0.054, 4.1, n)
        want = hasenbusch_masses(0.054, 4.1, n)
        assert all(abs(g - w) <= 1e-15 * w for g, w in zip(got, want))
    out = (ctypes.c_double * 2)()
    assert lib.hub_hasenbusch_masses(0.5, 0.1, 2, out) == b.HUB_ERR_ARG
    assert lib.hub_hasenbusch_masses(0.1, 0.5, 0, out) == b.HUB_ERR_ARG
    assert lib.hub_solve_multishift(None, None, None, None, 1, None, None, None, None, None, None) == b.HUB_ERR_ARG


def test_create_without_device_reports_hip_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_1804_07195_amd import binding as b
    h = ctypes.c_void_p()
    assert lib.hub_create(ctypes.byref(h), 0, 0) == b.HUB_ERR_HIP
    assert len(lib.hub_last_error()) > 0


def test_header_is_plain_c(lib, tmp_path):
    """include/hub.h compiles as C99 next to the HIP runtime header, and a C program
    that takes the address of every declared entry point links against libhub.so and
    runs its host-only call (no device is touched)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    names = declared_functions()
    src = tmp_path / "abi.c"
    src.write_text(
        '#include "hub.h"\n#include <stdio.h>\n'
        "int main(void) {\n"
        "  void* fns[] = {" + ", ".join(f"(void*){n}" for n in names) + "};\n"
        "  hub_solve_opts o;\n  hub_default_opts(&o);\n"
        '  printf("%d %d %d\\n", (int)(sizeof(fns) / sizeof(fns[0])), o.restart_m, fns[0] != 0);\n'
        "  return 0;\n}\n")
    exe = tmp_path / "abi"
    libdir = os.path.dirname(LIB)
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
                        "-I" + os.path.join(ROOT, "include"), "-I/opt/rocm/include", str(src), "-o", str(exe),
                        "-L" + libdir, "-lhub", "-Wl,-rpath," + libdir], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == [str(len(names)), "10", "1"]
