"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates parameters and workspace sizes before any
device call (no GPU needed)."""

import ctypes
import os
import re

import pytest

from paper_1511_08463_amd import fracture, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "fracture.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fracture_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = fracture.load_library()
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(fracture.EXPORTS) == declared


def test_header_constants_match_the_binding():
    """Every FRACTURE_* integer constant of the header has the same value in
    the Python binding (error codes, loads, modes, operator and kernel ids,
    failed-step stages)."""
    src = open(os.path.join(ROOT, "include", "fracture.h")).read()
    defs = dict((k, int(v)) for k, v in re.findall(r"#define\s+(FRACTURE_[A-Z0-9_]+)\s+(-?\d+)\b", src))
    assert len(defs) >= 30
    for k, v in defs.items():
        assert getattr(fracture, k) == v, k


def test_params_struct_matches_defaults():
    p = fracture.fracture_default_params(64, 32)
    assert (p.dim, p.nx, p.ny) == (2, 64, 32)
    assert p.model == fracture.FRACTURE_AT1 and p.omega == 1.0 and p.E == 1.0 and p.nu == 0.3
    assert p.k_ell == 1e-6 and p.cheb_degree == 2


def test_workspace_size_and_validation():
    p = fracture.make_params(**workloads.tension(64, 0.05))
    ws = fracture.fracture_workspace_bytes(p)
    N = 65 * 65
    assert ws > 40 * N * 8            # state, Krylov and multigrid vectors
    assert ws < 200 * N * 8
    big = fracture.make_params(**workloads.tension(2048, 4 / 2048))
    assert fracture.fracture_workspace_bytes(big) > 16 * ws
    # out-of-range parameters and empty or inverted meshes are refused
    for bad in (dict(omega=0.0), dict(omega=2.0), dict(ell=0.0), dict(nu=0.5),
                dict(model=3), dict(nx=5), dict(cheb_degree=0), dict(nx=0), dict(ny=0),
                dict(nx=-4), dict(lx=0.0), dict(ly=-1.0), dict(E=0.0), dict(Gc=0.0),
                dict(k_ell=-1.0), dict(max_am=0), dict(elem3d_min_nodes=-1)):
        q = fracture.make_params(**dict(workloads.tension(64, 0.05), **bad))
        assert fracture.fracture_workspace_bytes(q) == 0, bad


def test_create_rejects_bad_arguments_before_device_work():
    lib = fracture.load_library()
    p = fracture.make_params(**workloads.tension(64, 0.05))
    ws = fracture.fracture_workspace_bytes(p)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)           # never dereferenced: checks come first
    rc = lib.fracture_create(ctypes.byref(p), None, fake, ws - 1, None, ctypes.byref(h))
    assert rc == fracture.FRACTURE_ENOMEM
    rc = lib.fracture_create(ctypes.byref(p), None, ctypes.c_void_p((1 << 20) + 8), ws, None, ctypes.byref(h))
    assert rc == fracture.FRACTURE_EINVAL      # misaligned workspace
    p.omega = 2.5
    rc = lib.fracture_create(ctypes.byref(p), None, fake, ws, None, ctypes.byref(h))
    assert rc == fracture.FRACTURE_EINVAL
    assert lib.fracture_strerror(fracture.FRACTURE_ENOTCONV).decode().startswith("iteration limit")


def test_sizes():
    p = fracture.make_params(**workloads.tension(96, 0.05, nx=96, ny=80))
    n, d = fracture.fracture_sizes(p)
    assert n == 97 * 81 and d == 2 * n


def test_workload_recipes():
    p, notch, loads = workloads.config1()
    assert notch.sum() == 20 and notch.reshape(65, 65)[32, :20].all()
    assert loads[0] == pytest.approx(0.002) and loads[-1] == pytest.approx(0.02)
    p2, notch2, loads2, (y0, a) = workloads.config2()
    assert 0.1 <= y0 <= 0.4 and 0.1 <= a <= 0.4 and len(loads2) == 20
    assert notch2.sum() == int(round(a * 2048)) + 1


def test_every_gpu_test_shape_is_accepted():
    for nx, ny in [(8, 8), (16, 16), (32, 32), (48, 48), (64, 64), (96, 80), (64, 128), (2048, 2048)]:
        q = fracture.make_params(**workloads.tension(nx, 0.05, nx=nx, ny=ny))
        assert fracture.fracture_workspace_bytes(q) > 0, (nx, ny)


def test_3d_shapes_and_validation():
    from paper_1511_08463_amd import workloads as w
    p, loads = w.config3()
    q = fracture.make_params(**p)
    assert fracture.fracture_workspace_bytes(q) > 0
    n, d = fracture.fracture_sizes(q)
    assert n == 129 * 129 * 33 and d == 3 * n
    assert abs(w.thermal_dtc(p) - 2.049) < 1e-3 and len(loads) == 15
    assert abs(loads[-1] - 16 * w.thermal_dtc(p)) < 1e-12
    for shape in [(4, 4, 2), (12, 10, 6), (70, 4, 2), (32, 8, 4), (16, 8, 4)]:
        q = fracture.make_params(**w.thermal(*shape))
        assert fracture.fracture_workspace_bytes(q) > 0, shape
    # ORAM-N in 3D: the Newton block vectors [u_x | u_y | u_z | alpha] (4 N)
    # add to the workspace
    nw = fracture.make_params(**dict(w.thermal(16, 8, 4), newton=1))
    assert (fracture.fracture_workspace_bytes(nw)
            > fracture.fracture_workspace_bytes(fracture.make_params(**w.thermal(16, 8, 4)))
            + 7 * 4 * 17 * 9 * 5 * 8)
    bad = fracture.make_params(**dict(w.thermal(16, 8, 4), load_kind=0))
    assert fracture.fracture_workspace_bytes(bad) == 0


def test_deflation_parameters():
    """Crack-aware deflation: documented defaults, rejected combinations and
    the workspace it adds (three node-sized integer arrays and the small
    coarse-space buffers); the fragment entry points reject a null handle
    before any device work."""
    p = fracture.fracture_default_params(64, 64)
    assert (p.deflate, p.deflate_theta, p.deflate_min_nodes, p.deflate_max_fragments) == (0, 0.5, 64, 8)
    base = workloads.tension(64, 0.05)
    plain = fracture.fracture_workspace_bytes(fracture.make_params(**base))
    defl = fracture.fracture_workspace_bytes(fracture.make_params(**dict(base, deflate=1)))
    assert defl >= plain + 3 * 65 * 65 * 4
    for bad in (dict(deflate=2), dict(deflate=1, precision=fracture.FRACTURE_MIXED),
                dict(deflate=1, deflate_theta=0.0), dict(deflate=1, deflate_theta=1.5),
                dict(deflate=1, deflate_min_nodes=0), dict(deflate=1, deflate_max_fragments=0),
                dict(deflate=1, deflate_max_fragments=9)):
        q = fracture.make_params(**dict(base, **bad))
        assert fracture.fracture_workspace_bytes(q) == 0, bad
    th = workloads.thermal(16, 16, 4)
    assert fracture.fracture_workspace_bytes(fracture.make_params(**th)) > 0
    assert fracture.fracture_workspace_bytes(fracture.make_params(**dict(th, deflate=1))) == 0
    lib = fracture.load_library()
    n = ctypes.c_int()
    assert lib.fracture_fragments(None, ctypes.byref(n), None) == fracture.FRACTURE_EINVAL
    E = (ctypes.c_double * 576)()
    assert lib.fracture_deflation_matrix(None, ctypes.byref(n), E) == fracture.FRACTURE_EINVAL


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message before
    touching a device."""
    import json
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 2
    msg = json.loads(out.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_energy_noalloc_rejects_before_device_work():
    """NULL pointers, bad parameters and 3D meshes beyond the static scratch
    are refused before anything touches a device."""
    lib = fracture.load_library()
    fake = ctypes.c_void_p(1 << 20)           # never dereferenced: checks come first
    p = fracture.make_params(**workloads.tension(64, 0.05))
    rc = lib.fracture_energy_noalloc(ctypes.byref(p), 0.1, None, fake, None, fake)
    assert rc == fracture.FRACTURE_EINVAL
    rc = lib.fracture_energy_noalloc(ctypes.byref(p), float("nan"), fake, fake, None, fake)
    assert rc == fracture.FRACTURE_EINVAL
    p.nu = 0.5
    rc = lib.fracture_energy_noalloc(ctypes.byref(p), 0.1, fake, fake, None, fake)
    assert rc == fracture.FRACTURE_EINVAL
    # 3D: 6 tetrahedra x 8 bytes per hexahedron must fit in 32 MiB
    q = fracture.make_params(**workloads.thermal(128, 128, 64))
    rc = lib.fracture_energy_noalloc(ctypes.byref(q), 1.0, fake, fake, None, fake)
    assert rc == fracture.FRACTURE_ESCRATCH
    assert "scratch" in lib.fracture_strerror(fracture.FRACTURE_ESCRATCH).decode()


def test_bench_accepts_the_drivers_command():
    """`bench.py --gpus 1 --steps 20 --warmup 5` is a valid request: all 20
    load steps are timed, the warm-up runs on a separate instance."""
    import json
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "1", "--steps", "20",
                          "--warmup", "5", "--dry-run"], capture_output=True, text=True, timeout=120,
                         cwd=ROOT)
    assert out.returncode == 0, out.stderr
    pl = json.loads(out.stdout.strip().splitlines()[-1])["plan"]
    assert pl["timed_steps"] == list(range(1, 21))
    assert pl["warmup_steps"] == [1, 2, 3, 4, 5]
    assert "separate" in pl["warmup_instance"]
    assert pl["legs"][0] == "fp64" and "mixed" in pl["legs"]
    # the default run is the same plan with one warm-up step
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--dry-run"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert out.returncode == 0
    assert json.loads(out.stdout.strip().splitlines()[-1])["plan"]["timed_steps"] == list(range(1, 21))
