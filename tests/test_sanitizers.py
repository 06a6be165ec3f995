"""Host-side sanitizers: the C oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer runs every one of its entry points (filter and
its transpose, SIMP, assembly, products, CG, energies, tensor,
sensitivities, OC update) over small and odd cells, design iterations with
the governor included, without a report."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r"""
import numpy as np
import oracle as O
import synth
assert O.num_threads() >= 1
K = O.element_matrix()
for n in (3, 5, 6):
    rho = synth.smoothed_noise(n, 0.1, 0.9, 40 + n)
    for r in (0.0, 1.5, 2.5):
        f = O.density_filter(rho, r)
        O.density_filter_T(f, r)
    prm = O.Params(tol=1e-10)
    h = O.homogenize(rho, prm)
    A = O.assemble(O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal))
    x = np.random.default_rng(n).standard_normal((n, n, n))
    A.matvec(x)
    O.cg_fixed(A, O.macro_loads(O.simp(O.density_filter(rho, prm.rfilter), prm.k0, prm.kmin, prm.penal))[0], 5)
    w6 = 2.0 * (np.asarray(h["kappa"]) - np.array([0.3, 0.2, 0.1, 0.0, 0.0, 0.0]))
    s = O.sensitivities(h, w6, prm)
    O.oc_update(rho, s, 0.4)
    O.run(rho, [0.3, 0.2, 0.1, 0.0, 0.0, 0.0], 0.5, 2, prm)
print("oracle under sanitizers: ok")
"""


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as B
    try:
        asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("no gcc")
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no AddressSanitizer runtime")
    lib = B.build_sanitized(str(tmp_path / "liboracle_san.so"))
    env = dict(os.environ, LD_PRELOAD=asan, OTM_ORACLE_LIB=lib, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    out = subprocess.run([sys.executable, "-c", SCRIPT], env=env, capture_output=True, text=True, timeout=600)
    report = out.stdout + out.stderr
    assert out.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "oracle under sanitizers: ok" in out.stdout


HOST_SCRIPT = r"""
import ctypes, sys
import numpy as np
import paper_2405_19991_amd._native as N
N.LIBPATH = sys.argv[1]
L = N.lib()
assert b"gfx950" in L.otm_version()
s, o, g = N.default_options()
def problem(**kw):
    p = N.Problem()
    p.n, p.k0, p.kmin, p.penal, p.filter_radius, p.vf = 8, 1.0, 1e-3, 3.0, 1.5, 0.3
    for k, v in kw.items():
        setattr(p, k, v)
    return p
h = ctypes.c_void_p()
for kw in (dict(n=2), dict(n=2000), dict(kmin=0.0), dict(penal=0.5), dict(vf=1.5), dict(filter_radius=float("nan"))):
    p = problem(**kw)
    rc = L.otm_create(ctypes.byref(p), ctypes.byref(s), ctypes.byref(o), ctypes.byref(g), None, ctypes.byref(h))
    assert rc == N.OTM_EINVAL, kw
for kind in range(5):
    for n in (4, 7, 16, 33):
        out = np.empty(n ** 3)
        assert L.otm_init_density(n, kind, 0.3, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 0
for code in range(-8, 3):
    L.otm_strerror(code)
arr = (N.Problem * 2)(problem(), problem(n=9))
assert L.otm_batch_create(arr, 2, None, None, None, None, ctypes.byref(h)) == N.OTM_EINVAL
print("engine host paths under sanitizers: ok")
"""

# host code only: the device code is built as usual
HOST_SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer"


def test_engine_host_paths_under_sanitizers(tmp_path):
    """The library's host code built with AddressSanitizer and
    UndefinedBehaviorSanitizer (device code unchanged) runs the calls that
    need no GPU -- problem validation, initial densities for every kind and
    odd sizes, status strings, batch validation -- without a report."""
    import glob
    sys.path.insert(0, ROOT)
    from paper_2405_19991_amd import build as b
    runtime = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not runtime or not os.path.exists(hipcc):
        pytest.skip("no clang sanitizer runtime or hipcc")
    lib = str(tmp_path / "libopentm_san.so")
    flags = [f for f in b.FLAGS if f != "-O3"] + ["-O1", "-g", "-shared-libsan"] + HOST_SANITIZE.split()
    subprocess.run([hipcc, *flags, "-I", os.path.join(ROOT, "include"), "-I", b.CSRC,
                    *[os.path.join(b.CSRC, s) for s in b.SOURCES], "-o", lib], check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=runtime[-1], PYTHONPATH=ROOT, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([sys.executable, "-c", HOST_SCRIPT, lib], env=env, capture_output=True, text=True, timeout=600)
    report = out.stdout + out.stderr
    assert out.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "engine host paths under sanitizers: ok" in out.stdout
