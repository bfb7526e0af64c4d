"""The C ABI library loads and exports every entry point include/vklb.h
declares, and rejects invalid arguments before touching the GPU (no GPU)."""
import ctypes
import math
import os
import re

import pytest

from paper_2608_04283_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "vklb.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vklb_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def vk():
    from paper_2608_04283_amd import vklb
    vklb.lib()
    return vklb


def test_library_exports_every_declared_symbol(vk):
    L = vk.lib()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(vk.EXPORTED)


def test_workspace_bytes(vk):
    P = I.sod(65536)
    b64 = vk.workspace_bytes(P, "fp64")
    b32 = vk.workspace_bytes(P, "fp32")
    pop = 3 * 3 * 65536
    # two population buffers + FP64 staging of U, plus small state/partials
    assert b64 >= 2 * pop * 8 + 3 * 65536 * 8 and b64 < 2 * pop * 8 + 3 * 65536 * 8 + (1 << 20)
    # FP32 sizes for its largest basis: one more slot for the low part of U
    assert b32 >= 2 * (pop + 3 * 65536) * 4 + 3 * 65536 * 8 and b32 < b64
    bad = I.sod(10).with_(dim=2)
    assert vk.workspace_bytes(bad.with_(n=(10, 0)), "fp64") == 0


def create(vk, P, precision="fp64", **over):
    sysd, lat, grid, speed, eq, bc = vk._structs(P)
    for k, v in over.items():
        if k in ("omega", "lat"):
            continue
        obj, field = k.split(".")
        setattr({"sys": sysd, "grid": grid, "speed": speed, "eq": eq}[obj], field, v)
    if "lat" in over:
        lat = over["lat"]
    h = ctypes.c_void_p()
    r = vk.lib().vklb_create(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed),
                             over.get("omega", P.omega), bc, ctypes.byref(eq), vk.PRECISIONS[precision], None, None,
                             0, None, ctypes.byref(h))
    return r, vk.lib().vklb_last_error(None).decode()


@pytest.mark.parametrize("over,needle", [
    ({"omega": 0.0}, "omega"),
    ({"omega": 2.5}, "omega"),
    ({"speed.nu": 1.5}, "nu"),
    ({"speed.nu": 0.0}, "nu"),
    ({"eq.c": -0.1}, "c must"),
    ({"eq.k": -1.0}, "k must"),
    ({"sys.gamma": 1.0}, "gamma"),
    ({"eq.set": 3}, "equilibrium set"),
])
def test_invalid_arguments_rejected(vk, over, needle):
    r, msg = create(vk, I.sod(100), **over)
    assert r == vk.ERR_ARG and needle in msg


@pytest.mark.parametrize("prec,basis", [("fp64", 3), ("fp32", 4), ("fp64", -1)])
def test_invalid_basis_rejected(vk, prec, basis):
    """Basis is checked before any device call, so this runs without a GPU."""
    P = I.sod(100)
    sysd, lat, grid, speed, eq, bc = vk._structs(P)
    opt = vk.Options(basis, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    r = vk.lib().vklb_create(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed), P.omega, bc,
                             ctypes.byref(eq), vk.PRECISIONS[prec], ctypes.byref(opt), None, 0, None, ctypes.byref(h))
    assert r == vk.ERR_ARG and "basis" in vk.lib().vklb_last_error(None).decode()


def test_characteristic_boundary_scope(vk):
    """Characteristic boundaries (Sec. 3.3) are provided in 1D for every
    system; 2D grids are rejected as unsupported, a one-cell grid as invalid
    (the 1D MHD request passes validation and stops only at the missing
    device buffer)."""
    ch = ("characteristic", "characteristic")
    r, msg = create(vk, I.quadrants(16, steps=1).with_(bc=ch))
    assert r == vk.ERR_UNSUPPORTED and "characteristic" in msg
    r, msg = create(vk, I.brio_wu(64).with_(bc=ch))
    assert r != vk.ERR_UNSUPPORTED and "characteristic" not in msg
    r, msg = create(vk, I.sod(1).with_(bc=ch))
    assert r == vk.ERR_ARG and "2 cells" in msg


def test_tune_rejects_bad_step_count(vk):
    """Argument checks of vklb_tune come before any device call."""
    import numpy as np
    P = I.sod(100)
    sysd, lat, grid, speed, eq, bc = vk._structs(P)
    U0 = np.ascontiguousarray(P.U0)
    best = vk.Options()
    r = vk.lib().vklb_tune(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed), P.omega, bc,
                           ctypes.byref(eq), vk.PRECISIONS["fp32"], None, vk._dp(U0), 0, None, ctypes.byref(best),
                           None)
    assert r == vk.ERR_ARG


def test_size_limits(vk):
    """Empty grids are invalid; grids beyond 2^31 - 1 cells (32-bit cell
    indices on the device) are rejected as unsupported; the largest accepted
    grid reports its workspace size."""
    P = I.sod(100)
    for n in ((0,), (-5,)):
        assert vk.workspace_bytes(P.with_(n=n), "fp32") == 0
        r, msg = create(vk, P.with_(n=n))
        assert r == vk.ERR_ARG and "empty" in msg
    Q = I.quadrants(16, steps=1)
    big = Q.with_(n=(65536, 32768), hi=(2.0, 1.0))   # 2^31 cells: one too many
    assert vk.workspace_bytes(big, "fp32") == 0
    r, msg = create(vk, big)
    assert r == vk.ERR_UNSUPPORTED and "too large" in msg
    ok = Q.with_(n=(65535, 32768), hi=(65535 / 32768, 1.0))  # < 2^31 cells
    b = vk.workspace_bytes(ok, "fp32")
    cells = 65535 * 32768
    assert b >= 2 * 6 * 4 * cells * 4   # two buffers of (Q + 1) * p FP32 planes


def test_2d_rows_padded_to_64_cells(vk):
    """2D population buffers hold each row in a multiple of 64 cells (so a
    wavefront's row segment is one aligned run whatever the side), while the
    FP64 staging of U keeps the natural nx * ny cells: a 65-column grid needs
    the population bytes of a 128-column one."""
    Q = I.quadrants(16, steps=1)
    def pop_bytes(nx, ny):
        b = vk.workspace_bytes(Q.with_(n=(nx, ny), hi=(nx / ny, 1.0)), "fp32")
        assert b > 0
        return b - Q.p * nx * ny * 8          # minus the FP64 staging of U
    assert abs(pop_bytes(65, 64) - pop_bytes(128, 64)) <= 4096
    assert pop_bytes(65, 64) > pop_bytes(64, 64) + 2 * 20 * 63 * 64 * 4 - 4096
    assert abs(pop_bytes(64, 64) - pop_bytes(1, 64)) <= 4096    # one column pads to 64


def test_lattice_grid_mismatch_and_dx_dy(vk):
    r, msg = create(vk, I.sod(100), lat=1)
    assert r == vk.ERR_ARG and "lattice" in msg
    P = I.quadrants(16, steps=1).with_(n=(16, 8))
    r, msg = create(vk, P)
    assert r == vk.ERR_ARG and "dx == dy" in msg


def test_status_strings(vk):
    L = vk.lib()
    assert L.vklb_status_str(0) == b"ok"
    assert L.vklb_status_str(vk.ERR_NONPHYSICAL) == b"non-physical state"


def test_product_path_never_loads_the_oracle():
    """The package sources import nothing from oracle/ and read nothing from it."""
    pkg = os.path.join(ROOT, "paper_2608_04283_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".inc", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                for bad in ("import oracle", "from oracle", "oracle/", "oracle.py", "liboracle", "vklb_oracle"):
                    assert bad not in txt, (f, bad)


def test_plain_c_program_uses_the_abi(vk, tmp_path):
    """include/vklb.h is valid C99 (compiled with -pedantic, warnings as
    errors), and a C program linked against the library gets the same
    answers as the binding for the calls that need no GPU."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lib_dir = os.path.dirname(vk.LIB_PATH)
    exe = str(tmp_path / "abi_check")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "c", "abi_check.c"), "-L", lib_dir, "-lvklb",
                    "-Wl,-rpath," + lib_dir, "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=60).stdout.splitlines()
    got = dict(line.split(" ", 1) for line in out)
    assert got["status"] == "non-physical state"
    assert int(got["workspace_fp64"]) == vk.workspace_bytes(I.sod(65536), "fp64")
    code, msg = got["create_bad_omega"].split(" ", 1)
    assert int(code) == vk.ERR_ARG and "omega" in msg
    assert got["solver_null"] == "1"


def test_options_binding_matches_header(vk):
    """The binding's vklb_options has the header's int fields in the header's order."""
    import re
    hdr = open(os.path.join(ROOT, "include", "vklb.h")).read()
    end = hdr.index("} vklb_options;")
    body = hdr[hdr.rindex("typedef struct {", 0, end):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\bint\s+(\w+)\s*;", body)
    assert fields == [f[0] for f in vk.Options._fields_]
    assert all(t is ctypes.c_int for _, t in vk.Options._fields_)


def run_static_raw(vk, P, precision="fp64", n_steps=10, U0=1, U=1, T=math.inf, **over):
    """vklb_run_static with fake device pointers: every case here is rejected
    before anything is enqueued, so the pointers are never used."""
    sysd, lat, grid, speed, eq, bc = vk._structs(P)
    for k, v in over.items():
        obj, field = k.split(".")
        setattr({"sys": sysd, "grid": grid, "speed": speed, "eq": eq}[obj], field, v)
    L = vk.lib()
    r = L.vklb_run_static(ctypes.byref(sysd), lat, ctypes.byref(grid), ctypes.byref(speed), P.omega, bc,
                          ctypes.byref(eq), vk.PRECISIONS[precision], T, n_steps,
                          ctypes.c_void_p(U0) if U0 else None, ctypes.c_void_p(U) if U else None, None, None)
    return r, L.vklb_last_error(None).decode()


@pytest.mark.parametrize("case,status,needle", [
    ({"U0": 0}, "ERR_ARG", "NULL"),
    ({"U": 0}, "ERR_ARG", "NULL"),
    ({"n_steps": -1}, "ERR_ARG", "n_steps"),
    ({"T": math.nan}, "ERR_ARG", "NaN"),
    ({"speed.nu": 1.5}, "ERR_ARG", "nu"),
    ({"grid.n": None}, "ERR_OOM", "static"),
])
def test_run_static_rejects_before_enqueueing(vk, case, status, needle):
    """The allocation-free entry point checks its arguments and the static
    workspace's size before it touches the GPU."""
    P = I.sod(1000)
    if "grid.n" in case:
        # Euler 1D FP64 at 2^21 cells needs ~170 MB, above the 64 MiB array
        P = I.sod(1 << 21)
        case = {}
        assert vk.workspace_bytes(P, "fp64") > vk.STATIC_BYTES
    r, msg = run_static_raw(vk, P, **case)
    assert r == getattr(vk, status) and needle in msg, (r, msg)
