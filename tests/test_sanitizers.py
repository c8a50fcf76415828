"""Host sanitizer runs (no GPU): the plan engine (plan.cpp, dispatch.cpp)
recompiled with AddressSanitizer and UndefinedBehaviorSanitizer on the host
side and linked with the already built kernel objects, and the C oracle built
the same way with gcc; each is driven in a child process with its runtime
preloaded through plan creation over many shapes, kinds, grids, chains,
placements, storage orders and offset widths, the address emulation
(pfft_validate_plan), batches and every argument-error path.  Any sanitizer
report fails the test."""
import glob
import os
import shutil
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_09536_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g1"]

PLAN_DRIVER = textwrap.dedent("""
    import ctypes, itertools, sys
    sys.path.insert(0, %(root)r)
    from paper_1804_09536_amd import _lib
    _lib.LIB_PATH = %(lib)r
    from paper_1804_09536_amd.plan import Plan
    lib = _lib.load()
    n = 0
    shapes = [((8, 12, 16), (2, 3)), ((5, 7, 6), (2, 3)), ((3, 2, 4), (4, 3)), ((16, 17, 18, 19), (2, 2, 2)),
              ((12, 10, 8), (4,)), ((33, 17, 24), (8, 4)), ((6, 5, 4, 7), (2, 2, 3)), ((64, 1, 8), (2, 1))]
    for (shape, grid), kind, place, tr in itertools.product(shapes, ("c2c", "r2c"), ("gather", "direct", "final"),
                                                           (False, True)):
        if kind == "r2c":
            shape = shape[:-1] + (2 * shape[-1],)
        try:
            p = Plan(shape, grid, kind=kind, placement=(place, "scatter"), transposed_out=tr, device="cpu")
        except _lib.PfftError:
            continue
        p.validate()
        p.set_tuning(tile_strided=2, xcd_order=1, wide_offsets=1)
        p.validate()
        p.set_tuning(tile_strided=5, xcd_order=0, wide_offsets=0, radix_alt=3)
        p.validate()
        n += 1
    for path in ("unfused", "pack_realign"):
        Plan((8, 12, 16), (2, 3), path=path, destroy_input=True, device="cpu").validate()
    Plan((8, 12, 10), (4,), chain=[(0, 2)], device="cpu").validate()
    Plan((8, 12, 16), (2, 3), kind="r2r", r2r=("dct2", "dst2", "dct2"), device="cpu").validate()
    Plan((4, 4, 4099), (2, 2), device="cpu").validate()          # Bluestein tables
    for args in [((16, 0, 16), (2, 2)), ((16, 16), (2, 2)), ((4, 4, 10247), (2, 2))]:
        try:
            Plan(*args, device="cpu")
        except _lib.PfftError:
            pass
    plans = [Plan((8, 12, 16), (2, 3), device="cpu"), Plan((6, 8, 10), (2,), device="cpu")]
    h = ctypes.c_void_p()
    arr = (ctypes.c_void_p * 3)(plans[0]._h.value, plans[1]._h.value, plans[0]._h.value)
    assert lib.pfft_batch_create(ctypes.byref(h), 3, arr) == 0
    assert lib.pfft_batch_destroy(h) == 0
    v = ctypes.c_void_p
    assert lib.pfft_forward(None, None, None, None, None) == -1
    assert lib.pfft_redistribute(plans[0]._h, 0, 5, v(1 << 20), v(1 << 24), None) == -1
    assert lib.pfft_weighted_energy(0, -1, v(4096), v(4096), v(4096), v(4096), None) == -1
    print("plans", n)
""")

ORACLE_DRIVER = textwrap.dedent("""
    import sys
    sys.path.insert(0, %(root)r)
    import numpy as np
    import oracle.core as core
    core._LIB_PATH = %(lib)r
    import oracle
    rng = np.random.default_rng(0)
    for shape, grid, kind in [((6, 5, 4), (2, 3), "c2c"), ((4, 6, 5, 3), (2, 2, 3), "c2c"), ((6, 8, 10), (2, 3), "r2c"),
                              ((3, 2, 4), (4, 3), "c2c"), ((12, 10, 8), (4,), "c2c")]:
        ch = oracle.Chain.paper(shape, grid, kind=kind)
        n = int(np.prod(shape))
        u = rng.standard_normal(n) + (1j * rng.standard_normal(n) if kind == "c2c" else 0)
        y = oracle.forward(ch, u)
        oracle.backward(ch, y)
        oracle.adjoint_forward(ch, y)
        oracle.adjoint_backward(ch, u)
    ch = oracle.Chain.paper((4, 6, 5), (2, 3))
    x = rng.standard_normal(120) + 1j * rng.standard_normal(120)
    for li in range(len(ch.dirs) - 1):
        oracle.redistribute(x, ch.layout(li), ch.layout(li + 1))
        oracle.redistribute_pairs(x, ch.layout(li), ch.layout(li + 1))
    oracle.bruteforce_dftn(x.reshape(4, 6, 5), -1, 1.0)
    oracle.dft_bins(x.reshape(4, 6, 5), [(1, 2, 3), (0, 0, 0)], -1, 1.0)
    for n in (1, 7, 12, 127, 384, 1000):
        oracle.dft1(rng.standard_normal(n) + 0j, -1)
    print("oracle ok")
""")


def _run(code, env):
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    return report


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_plan_engine_under_asan_ubsan(tmp_path):
    from paper_1804_09536_amd import build as pbuild
    rt = _clang_asan_runtime()
    objs = [os.path.join(BUILD, os.path.splitext(f)[0] + ".o") for f in pbuild.sources()]
    if rt is None or not all(os.path.exists(o) for o in objs):
        pytest.skip("needs the built kernel objects and clang's ASan runtime")
    san_objs = {}
    for src in ("plan.cpp", "dispatch.cpp"):
        out = str(tmp_path / (src + ".o"))
        cmd = [pbuild.HIPCC] + pbuild.COMMON + ["-x", "hip"] + pbuild.DEVICE + \
              [a for f in SAN for a in ("-Xarch_host", f)] + ["-c", os.path.join(CSRC, src), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        san_objs[src] = out
    link = [san_objs.get(os.path.basename(o)[:-2] + ".cpp", o) if os.path.basename(o) in ("plan.o", "dispatch.o")
            else o for o in objs]
    lib = str(tmp_path / "libpfft_asan.so")
    r = subprocess.run([pbuild.HIPCC, "-shared", "-fPIC", "--offload-arch=" + pbuild.ARCH, "-o", lib] + link +
                       ["-Xarch_host", "-fsanitize=address,undefined", "-shared-libasan"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = _run(PLAN_DRIVER % {"root": ROOT, "lib": lib}, env)
    assert "plans" in out


def test_oracle_under_asan_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    asan = subprocess.run([gcc, "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run([gcc, "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    if not (os.path.isabs(asan) and os.path.isabs(ubsan)):
        pytest.skip("gcc sanitizer runtimes not found")
    lib = str(tmp_path / "liboracle_asan.so")
    src = os.path.join(ROOT, "oracle", "oracle.c")
    r = subprocess.run([gcc, "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-D_DEFAULT_SOURCE"] + SAN +
                       ["-o", lib, src, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, LD_PRELOAD=asan + ":" + ubsan, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    out = _run(ORACLE_DRIVER % {"root": ROOT, "lib": lib}, env)
    assert "oracle ok" in out
