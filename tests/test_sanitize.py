"""CPU sanitizer build: the library's host assembly and solver copy
(assemble.cpp) and the oracle (femoracle.c), compiled with g++/gcc and
-fsanitize=address,undefined into one driver (tests/sanitize/san_driver.cpp),
run on 2D/3D, P1-P4, jittered meshes.  The host assembly leaves its large
arrays uninitialised and fills them with parallel loops and sorts; an
out-of-bounds access or undefined behaviour there (or in the oracle) aborts
the driver.  The driver also checks the library's assembly and solver copies
against the oracle, and the oracle's PCG against its own Eq. (2) residual."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import meshgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_05413_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="needs gcc/g++")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    cxx = ["g++", "-std=c++17"] + SAN + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                        "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
    objs = []
    for src in (os.path.join(CSRC, "assemble.cpp"), os.path.join(ROOT, "tests", "sanitize", "san_driver.cpp")):
        o = str(d / (os.path.basename(src) + ".o"))
        subprocess.check_call(cxx + ["-c", src, "-o", o])
        objs.append(o)
    o = str(d / "femoracle.o")
    subprocess.check_call(["gcc", "-std=c11"] + SAN + ["-c", os.path.join(ROOT, "oracle", "femoracle.c"), "-o", o],
                          stderr=subprocess.DEVNULL)
    objs.append(o)
    exe = str(d / "san_driver")
    subprocess.check_call(["g++"] + SAN + ["-o", exe] + objs + ["-lpthread", "-lm"])
    return exe, d


def _write_mesh(path, mesh):
    coords = np.ascontiguousarray(mesh["coords"], dtype=np.float64)
    cells = np.ascontiguousarray(mesh["cells"], dtype=np.int32)
    bnd = np.ascontiguousarray(mesh["on_boundary"], dtype=np.uint8)
    with open(path, "wb") as f:
        f.write(np.array([coords.shape[1], coords.shape[0], cells.shape[0]], dtype=np.int64).tobytes())
        f.write(coords.tobytes())
        f.write(cells.tobytes())
        f.write(bnd.tobytes())


@pytest.mark.parametrize("dim,m,jit,order", [(2, 24, 0.3, 1), (2, 13, 0.25, 2), (2, 9, 0.3, 3), (2, 8, 0.2, 4),
                                             (3, 8, 0.3, 1), (3, 6, 0.3, 2), (2, 40, 0.0, 1)])
def test_host_assembly_and_oracle_under_asan_ubsan(driver, dim, m, jit, order):
    exe, d = driver
    path = str(d / ("mesh_%d_%d_%d.bin" % (dim, m, order)))
    _write_mesh(path, meshgen.make_mesh(dim, m, jit, 70 + m))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, path, str(order)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "0 failure(s)" in r.stdout
