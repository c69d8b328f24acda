"""CPU checks of the C ABI: the library loads, exports every symbol the header
declares, and rejects invalid descriptors before touching the device."""
import ctypes
import os
import subprocess
import sys

import pytest

from paper_2105_01722_amd import gdw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_header_symbol_is_exported():
    names = gdw.header_symbols()
    assert "gdw_create" in names and "gdw_run" in names
    out = subprocess.run(["nm", "-D", "--defined-only", gdw.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(gdw.lib, n)


def test_version_and_no_error():
    assert "gfx950" in gdw.gdw_version()
    assert isinstance(gdw.lib.gdw_last_error(), bytes)


def _desc(**kw):
    d = gdw.gdw_desc()
    d.nx, d.ny, d.N, d.p = 4, 4, 8, 3
    d.x0 = d.y0 = 0.0
    d.Lx = d.Ly = 1.0
    d.c2 = 1.0
    d.flux = gdw.GDW_FLUX_CENTRAL
    d.xi = 1.0
    d.precision = gdw.GDW_FP64
    d.solver = gdw.GDW_SOLVE_AUTO
    for k, v in kw.items():
        if k == "bc":
            for i, b in enumerate(v):
                d.bc[i] = b
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,status", [
    (dict(p=4), gdw.GDW_EINVAL),
    (dict(p=0), gdw.GDW_EINVAL),
    (dict(N=2, p=3), gdw.GDW_EINVAL),
    (dict(nx=0), gdw.GDW_EINVAL),
    (dict(Lx=-1.0), gdw.GDW_EINVAL),
    (dict(c2=0.0), gdw.GDW_EINVAL),
    (dict(c2=float("nan")), gdw.GDW_EINVAL),
    (dict(flux=7), gdw.GDW_EINVAL),
    (dict(flux=gdw.GDW_FLUX_UPWIND, xi=0.0), gdw.GDW_EINVAL),
    (dict(precision=9), gdw.GDW_EINVAL),
    (dict(N=32), gdw.GDW_EINVAL),
    (dict(solver=gdw.GDW_SOLVE_FDM, coeff_variable=1), gdw.GDW_EINVAL),
    (dict(solver=gdw.GDW_SOLVE_FDM, mapped=1), gdw.GDW_EINVAL),
    (dict(coeff_variable=1, N=12, p=9), gdw.GDW_EUNSUPPORTED),
    (dict(mapped=1, pcg_rtol=float("nan")), gdw.GDW_EINVAL),
    (dict(bc=(7, 7, 0, 0)), gdw.GDW_EINVAL),
    (dict(bc=(gdw.GDW_BC_DIRICHLET, gdw.GDW_BC_PERIODIC, 0, 0)), gdw.GDW_EINVAL),
    (dict(bc=(0, 0, gdw.GDW_BC_PERIODIC, gdw.GDW_BC_NEUMANN)), gdw.GDW_EINVAL),
    (dict(bc=(gdw.GDW_BC_DIRICHLET, gdw.GDW_BC_NEUMANN, 3, 0), coeff_variable=1), gdw.GDW_EINVAL),
])
def test_invalid_descriptors_rejected_on_host(kw, status):
    """Validation happens before any device call, so it runs without a GPU."""
    ctx = ctypes.c_void_p()
    st = gdw.lib.gdw_create(ctypes.byref(_desc(**kw)), ctypes.byref(ctx))
    assert st == status
    assert ctx.value is None
    assert gdw.lib.gdw_last_error()


def test_null_arguments_rejected():
    assert gdw.lib.gdw_create(None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_run(None, 0.1, 1, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_set_state(None, None, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_get_state(None, None, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_energy(None, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_get_stats(None, None, None) == gdw.GDW_EINVAL
    gdw.lib.gdw_destroy(None)


def test_product_path_does_not_import_oracle():
    """The package never imports the oracle (the oracle is test infrastructure)."""
    pkg = os.path.join(ROOT, "paper_2105_01722_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_one_hip_runtime_in_the_process():
    """Importing the binding first (before anything else imports torch) must leave one HIP
    runtime and one HSA runtime in the process: torch's, which owns the tensors the library
    is handed.  Two HSA runtimes in one process make the second report no GPU."""
    code = ("from paper_2105_01722_amd import gdw\n"
            "import torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps')\n"
            "        if 'libamdhip64' in l or 'libhsa-runtime64' in l}\n"
            "print('\\n'.join(sorted(libs)))\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    libs = out.stdout.split()
    assert sum("libamdhip64" in l for l in libs) == 1, libs
    assert sum("libhsa-runtime64" in l for l in libs) == 1, libs


@pytest.mark.parametrize("args", [(0, 16, 8, 1, 64), (64, 0, 8, 1, 64), (64, 16, 0, 1, 64),
                                  (64, 16, 8, 1, 0), (64, 100000, 8, 1, 64)])
def test_mlp_create_rejects_bad_sizes(args):
    h = ctypes.c_void_p()
    assert gdw.lib.gdw_mlp_create(*args, ctypes.byref(h)) == gdw.GDW_EINVAL
    assert h.value is None


def test_mlp_and_precond_null_arguments():
    assert gdw.lib.gdw_mlp_get_params(None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_mlp_forward(None, None, 1, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_mlp_train(None, None, None, 1, 1, 1, ctypes.c_float(1e-3), None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_precond_data(None, None, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_set_precond_mlp(None, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_set_coeff(None, None, None, None, None) == gdw.GDW_EINVAL
    gdw.lib.gdw_mlp_destroy(None)


def test_batch_arguments_rejected_on_host():
    import ctypes
    from paper_2105_01722_amd import gdw
    h = ctypes.c_void_p()
    d = (gdw.gdw_desc * 1)(gdw.make_desc(2, 2, 8, 3))
    assert gdw.lib.gdw_batch_create(0, d, ctypes.byref(h)) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_create(5000, d, ctypes.byref(h)) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_create(1, None, ctypes.byref(h)) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_ctx(None, 0, ctypes.byref(h)) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_run(None, None, 1, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_tune(None, None, None) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_step_times(None, None, 0) == gdw.GDW_EINVAL
    assert gdw.lib.gdw_batch_plan(None) == b""
    gdw.lib.gdw_batch_destroy(None)


def test_bench_refuses_several_gpus_before_touching_a_device():
    """bench.py measures one GPU: --gpus N with N > 1 exits with status 2 and a message,
    before any device work (so this runs without a GPU)."""
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


def test_3d_requests_outside_the_box_path_are_refused():
    """3D runs on the constant-coefficient Cartesian path only, with (N + 1)^3 <= 1024;
    validation refuses the rest before any device work, and a batch refuses 3D members."""
    from paper_2105_01722_amd import gdw
    for kw, status in ((dict(solver="pcg"), gdw.GDW_EUNSUPPORTED),
                       (dict(coeff_variable=True), gdw.GDW_EUNSUPPORTED),
                       (dict(N=10), gdw.GDW_EUNSUPPORTED),
                       (dict(Lz=-1.0), gdw.GDW_EINVAL),
                       (dict(bcz=("dirichlet", "periodic")), gdw.GDW_EINVAL)):
        args = dict(nx=2, ny=2, N=8, p=3, nz=2)
        args.update(kw)
        d = gdw.make_desc(**args)
        with pytest.raises(gdw.GdwError) as ei:
            gdw.gdw_create(d)
        assert ei.value.status == status, (kw, ei.value)
    d = gdw.make_desc(nx=2, ny=2, N=8, p=3)
    d.dim = 4
    with pytest.raises(gdw.GdwError) as ei:
        gdw.gdw_create(d)
    assert ei.value.status == gdw.GDW_EINVAL
    with pytest.raises(gdw.GdwError) as ei:
        gdw.Batch([dict(nx=2, ny=2, N=8, p=3, nz=2)])
    assert ei.value.status == gdw.GDW_EUNSUPPORTED
