"""Host-side checks of the C ABI library (no GPU needed).

The library must load, export every function include/opentm_amd.h declares,
and reject invalid problems before touching a device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "opentm_amd.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(otm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2405_19991_amd import _native as N
    if not os.path.exists(N.LIBPATH):
        pytest.fail("libopentm_amd.so is not built; run __graft_entry__.build()")
    return N.lib()


def test_exports_match_header(L):
    from paper_2405_19991_amd import _native as N
    declared = header_functions()
    assert declared, "no functions parsed from the header"
    assert sorted(N.EXPORTED) == declared
    for name in declared:
        assert hasattr(L, name), name


def test_version_and_strerror(L):
    assert b"gfx950" in L.otm_version()
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert L.otm_strerror(code)
    assert L.otm_strerror(99) == b"unknown status"


def test_default_options_follow_paper_parameters(L):
    from paper_2405_19991_amd import _native as N
    s, o, g = N.default_options()
    assert (o.move, o.eta, o.rho_min) == (0.05, 0.5, 1e-3)
    assert (g.bound, g.decay, g.rebound, g.patience) == (1e-4, 0.8, 0.3, 5)
    assert s.precision == N.OTM_FP64 and s.tol > 0 and s.check_every >= 1


@pytest.mark.parametrize("field,value", [("n", 2), ("n", 2000), ("kmin", 0.0), ("kmin", 2.0), ("penal", 0.5),
                                         ("vf", 0.0), ("vf", 1.5), ("filter_radius", float("nan"))])
def test_create_rejects_invalid_problem(L, field, value):
    from paper_2405_19991_amd import _native as N
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 8, 1.0, 1e-3, 3.0, 1.5, 0.3
    setattr(p, field, value)
    h = ctypes.c_void_p()
    rc = L.otm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h))
    assert rc == N.OTM_EINVAL
    assert not h.value


def test_null_arguments(L):
    from paper_2405_19991_amd import _native as N
    assert L.otm_create(None, None, None, None, None, None) == N.OTM_EINVAL
    assert L.otm_apply_device(2, 0, 0, None, None, None, None) == N.OTM_EINVAL
    assert L.otm_last_error(None) == b"null context"
    b = ctypes.c_int64(-1)
    assert L.otm_device_bytes(None, ctypes.byref(b)) == N.OTM_EINVAL
    assert L.otm_batch_device_bytes(None, ctypes.byref(b)) == N.OTM_EINVAL
    assert b.value == -1
    # checkpoint calls: a null handle or an empty path is refused before any file or device access
    for fn in (L.otm_save_state, L.otm_load_state, L.otm_batch_save_state, L.otm_batch_load_state):
        assert fn(None, b"/nonexistent/state.otm") == N.OTM_EINVAL
        assert fn(None, None) == N.OTM_EINVAL
    assert L.otm_nn_load(None, b"/nonexistent/w.npy") == N.OTM_EINVAL


def test_batch_create_rejects_odd_or_bad_sizes(L):
    from paper_2405_19991_amd import _native as N
    arr = (N.Problem * 2)()
    for p in arr:
        p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 8, 1.0, 1e-3, 3.0, 1.5, 0.3
    arr[1].n = 9
    h = ctypes.c_void_p()
    assert L.otm_batch_create(arr, 2, None, None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    assert L.otm_batch_create(arr, 0, None, None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    assert L.otm_batch_last_error(None) == b"null batch"


@pytest.mark.parametrize("n,precision,variant,sweeps", [(10, 1, 0, 2), (4, 1, 0, 2), (7, 1, 0, 2), (10, 0, 0, 2),
                                                        (16, 1, 4, 2), (16, 0, 1, 2), (16, 1, 0, 0), (16, 1, 0, 9)])
def test_multigrid_options_rejected(L, n, precision, variant, sweeps):
    """The V-cycle needs n = m 2^j (m in {3, 4}, n >= 6), the two-pass
    iteration and 1..8 relaxation steps (either precision)."""
    from paper_2405_19991_amd import _native as N
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = n, 1.0, 1e-3, 3.0, 1.5, 0.3
    s, o, g = N.default_options()
    s.precision, s.kernel_variant, s.preconditioner, s.mg_sweeps = precision, variant, N.OTM_PRECOND_MG, sweeps
    h = ctypes.c_void_p()
    assert L.otm_create(ctypes.byref(p), ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    assert not h.value


def test_multigrid_coarse_sweeps_rejected(L):
    from paper_2405_19991_amd import _native as N
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 16, 1.0, 1e-3, 3.0, 1.5, 0.3
    s, o, g = N.default_options()
    assert (s.mg_sweeps, s.mg_coarse_sweeps) == (1, 2)
    s.precision, s.preconditioner = N.OTM_MIXED, N.OTM_PRECOND_MG
    h = ctypes.c_void_p()
    for bad in (-1, 9):
        s.mg_coarse_sweeps = bad
        assert L.otm_create(ctypes.byref(p), ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL


def test_batch_rejects_multigrid(L):
    from paper_2405_19991_amd import _native as N
    arr = (N.Problem * 1)()
    arr[0].n, arr[0].k0, arr[0].kmin, arr[0].penal, arr[0].filter_radius, arr[0].vf = 16, 1.0, 1e-3, 3.0, 1.5, 0.3
    s, o, g = N.default_options()
    s.preconditioner = N.OTM_PRECOND_MG
    h = ctypes.c_void_p()
    assert L.otm_batch_create(arr, 1, ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EUNSUPPORTED


def test_batch_precision_validation(L):
    """Mixed-precision batches run the fused iteration only; unknown
    precisions and a non-positive refresh threshold are invalid."""
    from paper_2405_19991_amd import _native as N
    arr = (N.Problem * 1)()
    arr[0].n, arr[0].k0, arr[0].kmin, arr[0].penal, arr[0].filter_radius, arr[0].vf = 16, 1.0, 1e-3, 3.0, 1.5, 0.3
    h = ctypes.c_void_p()
    for variant, code in ((1, N.OTM_EUNSUPPORTED), (2, N.OTM_EUNSUPPORTED), (5, N.OTM_EUNSUPPORTED),
                          (6, N.OTM_EINVAL)):
        s, o, g = N.default_options()
        s.precision, s.kernel_variant = N.OTM_MIXED, variant
        assert L.otm_batch_create(arr, 1, ctypes.byref(s), None, None, None, ctypes.byref(h)) == code
    s, o, g = N.default_options()
    s.precision = 7
    assert L.otm_batch_create(arr, 1, ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    s, o, g = N.default_options()
    s.precision, s.reliable_delta = N.OTM_MIXED, 0.0
    assert L.otm_batch_create(arr, 1, ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    s, o, g = N.default_options()
    s.stall_window = -1
    assert L.otm_batch_create(arr, 1, ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL


def _problem(N, n=8):
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = n, 1.0, 1e-3, 3.0, 1.5, 0.3
    for q, t in enumerate((0.3, 0.2, 0.1, 0.05, 0.05, 0.05)):
        p.target[q] = t
    return p


def test_objective_and_symmetry_validation(L):
    from paper_2405_19991_amd import _native as N
    h = ctypes.c_void_p()
    p = _problem(N)
    p.objective = 3
    assert L.otm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h)) == N.OTM_EUNSUPPORTED
    p = _problem(N)
    p.objective = N.OTM_OBJ_REL
    p.target[4] = 0.0  # the relative objective divides by every target component
    assert L.otm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    p = _problem(N)
    p.symmetry = 2
    assert L.otm_create(ctypes.byref(p), None, None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    arr = (N.Problem * 1)()
    arr[0] = _problem(N)
    arr[0].symmetry = N.OTM_SYM_CENTRAL
    assert L.otm_batch_create(arr, 1, None, None, None, None, ctypes.byref(h)) == N.OTM_EUNSUPPORTED


@pytest.mark.parametrize("field,value", [("patience", 0), ("stall_iters", 0), ("decay", 1.5), ("decay", -0.1),
                                         ("bound", float("nan")), ("dg_small", -1.0), ("rebound", float("inf"))])
def test_governor_options_rejected(L, field, value):
    """Adaptive volume bound options are checked before any device work, for
    single contexts and batches."""
    from paper_2405_19991_amd import _native as N
    p = _problem(N)
    s, o, g = N.default_options()
    setattr(g, field, value)
    h = ctypes.c_void_p()
    assert L.otm_create(ctypes.byref(p), None, None, ctypes.byref(g), None, ctypes.byref(h)) == N.OTM_EINVAL
    assert not h.value
    arr = (N.Problem * 1)()
    arr[0] = _problem(N)
    assert L.otm_batch_create(arr, 1, None, None, ctypes.byref(g), None, ctypes.byref(h)) == N.OTM_EINVAL
    b8 = (ctypes.c_double * 8)()
    assert L.otm_batch_get_governor(None, 0, b8) == N.OTM_EINVAL


def test_oc_noalloc_validates_before_any_device_call(L):
    """The allocation-free OC update rejects null buffers, sizes beyond
    4..1024, V* outside (0, 1], bad options and aliasing on the host, before
    it looks up its scratch or launches anything (fake non-null addresses are
    never dereferenced)."""
    from paper_2405_19991_amd import _native as N
    oc = N.OcOpts(0.05, 0.5, 1e-3)
    a, b, c, d = (ctypes.c_void_p(v) for v in (0x1000, 0x2000, 0x3000, 0x4000))
    f = L.otm_oc_update_noalloc
    assert f(16, None, b, 0.3, ctypes.byref(oc), c, None, None) == N.OTM_EINVAL
    assert f(16, a, None, 0.3, ctypes.byref(oc), c, None, None) == N.OTM_EINVAL
    assert f(16, a, b, 0.3, ctypes.byref(oc), None, None, None) == N.OTM_EINVAL
    assert f(16, a, b, 0.3, None, c, None, None) == N.OTM_EINVAL
    for n in (3, 1025, 4096):
        assert f(n, a, b, 0.3, ctypes.byref(oc), c, None, None) == N.OTM_EINVAL
    for v in (0.0, -0.1, 1.5, float("nan")):
        assert f(16, a, b, v, ctypes.byref(oc), c, None, None) == N.OTM_EINVAL
    for bad in (N.OcOpts(0.0, 0.5, 1e-3), N.OcOpts(0.05, 0.0, 1e-3), N.OcOpts(0.05, 0.5, 0.0),
                N.OcOpts(0.05, 0.5, 1.0)):
        assert f(16, a, b, 0.3, ctypes.byref(bad), c, None, None) == N.OTM_EINVAL
    assert f(16, a, b, 0.3, ctypes.byref(oc), b, None, None) == N.OTM_EINVAL  # out aliases sens
    assert f(16, a, b, 0.3, ctypes.byref(oc), c, a, None) == N.OTM_EINVAL    # lambda aliases rho
    assert f(16, a, b, 0.3, ctypes.byref(oc), c, c, None) == N.OTM_EINVAL    # lambda aliases out


def test_create_rejects_negative_stall_window(L):
    from paper_2405_19991_amd import _native as N
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 8, 1.0, 1e-3, 3.0, 1.5, 0.3
    s, o, g = N.default_options()
    assert s.stall_window == 0
    s.stall_window = -1
    h = ctypes.c_void_p()
    assert L.otm_create(ctypes.byref(p), ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
    assert not h.value


@pytest.mark.parametrize("move_min", [-1e-3, 0.06, float("nan")])
def test_create_rejects_bad_move_floor(L, move_min):
    """The adaptive OC move floor must lie in [0, move] (default move 0.05)."""
    from paper_2405_19991_amd import _native as N
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 8, 1.0, 1e-3, 3.0, 1.5, 0.3
    s, o, g = N.default_options()
    assert o.move_min == 0.0
    o.move_min = move_min
    h = ctypes.c_void_p()
    assert L.otm_create(ctypes.byref(p), None, ctypes.byref(o), None, None, ctypes.byref(h)) == N.OTM_EINVAL
    assert not h.value


def test_multigrid_smoother_rejected(L):
    from paper_2405_19991_amd import _native as N
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 16, 1.0, 1e-3, 3.0, 1.5, 0.3
    s, o, g = N.default_options()
    assert s.mg_smoother == N.OTM_MG_JACOBI
    s.precision, s.preconditioner, s.mg_smoother = N.OTM_MIXED, N.OTM_PRECOND_MG, 2
    h = ctypes.c_void_p()
    assert L.otm_create(ctypes.byref(p), ctypes.byref(s), None, None, None, ctypes.byref(h)) == N.OTM_EINVAL


def test_header_is_c_and_layouts_match_binding(L, tmp_path):
    """The public header compiles as C99 on its own; a C program linked
    against the library runs the host-only calls (version, default options,
    initial densities); and every public struct has the size and the field
    offsets of its ctypes mirror in the Python binding."""
    import shutil
    import subprocess
    from paper_2405_19991_amd import _native as N
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"otm_problem": N.Problem, "otm_solver_opts": N.SolverOpts, "otm_oc_opts": N.OcOpts,
               "otm_governor_opts": N.GovernorOpts, "otm_solve_stats": N.SolveStats,
               "otm_iter_record": N.IterRecord}
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "opentm_amd.h"', "int main(void) {"]
    cfield = {"lambda_": "lambda"}  # Python keywords carry a trailing underscore in the binding
    for cname, cls in structs.items():
        src.append(f'    printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            src.append(f'    printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cfield.get(fname, fname)}));')
    src += ['    printf("version %s\\n", otm_version());',
            "    otm_solver_opts s; otm_oc_opts o; otm_governor_opts g;",
            "    otm_default_options(&s, &o, &g);",
            '    printf("move %.3f\\n", o.move);',
            "    static double rho[8 * 8 * 8];",
            "    int rc = otm_init_density(8, OTM_INIT_P, 0.25, rho);",
            "    int solid = 0;",
            "    for (int i = 0; i < 512; ++i) solid += rho[i] > 0.5;",
            '    printf("init %d %d\\n", rc, solid);',
            "    return 0;", "}"]
    prog = tmp_path / "abi_check.c"
    prog.write_text("\n".join(src) + "\n")
    exe = tmp_path / "abi_check"
    libdir = os.path.dirname(N.LIBPATH)
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(prog),
                    "-L", libdir, "-lopentm_amd", "-Wl,-rpath," + libdir, "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = dict(line.split(" ", 1) for line in out if line)
    for cname, cls in structs.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, f"{cname}.{fname}"
    assert "gfx950" in got["version"]
    assert float(got["move"]) == 0.05
    rc, solid = map(int, got["init"].split())
    assert rc == 0 and solid == round(0.25 * 512)
