"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

Every library source is compiled with the sanitizers on its host side only
(the device code is unchanged), linked into a private copy of libasp.so, and
two host programs run against it on host-only plans:

* tests/host_plans.cpp: the plan builder (partition, auxiliary grids, PML
  tables, sizes, workspace estimates, argument checks) for 2D and 3D plans with
  equal and unequal widths, thin auxiliary PML and both 3D factorizations;
* tests/nd_emulation.cpp: the nested-dissection tree, front column lists and
  child maps, driving a complex-double multifrontal factor and solve of every
  slab on the CPU.

Any invalid access, leak or undefined behaviour aborts the program."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1504_04058_amd", "csrc")
INC = os.path.join(ROOT, "include")
# host-side sanitizers only: each -fsanitize applies to the host compilation
SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        pytest.skip("hipcc not available")
    return path


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, " ".join(cmd) + "\n" + res.stderr[-3000:]


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    hipcc = _hipcc()
    d = tmp_path_factory.mktemp("san")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I" + INC] + SAN
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".cpp", ".hip")))
    objs = [str(d / (os.path.basename(s) + ".o")) for s in srcs]
    with ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(lambda so: _run([hipcc, "-x", "hip", *flags, "-c", so[0], "-o", so[1]]),
                    zip(srcs, objs)))
    lib = str(d / "libasp.so")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-o", lib, *objs])
    exes = {}
    for name, extra in (("host_plans", []), ("nd_emulation", ["-I" + CSRC])):
        exe = str(d / name)
        _run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", *SAN,
              os.path.join(HERE, name + ".cpp"), "-o", exe, "-I" + INC, *extra,
              "-L" + str(d), "-lasp", "-Wl,-rpath," + str(d)])
        exes[name] = exe
    return exes


def test_plan_builder_under_sanitizers(sanitized):
    res = subprocess.run([sanitized["host_plans"]], capture_output=True, text=True, env=ENV,
                         timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert res.stdout.strip().endswith("ok (0 failures)")


@pytest.mark.parametrize("n,b,gamma,aux", [(11, 3, 3, 0), (17, 4, 4, 3)])
def test_nested_dissection_host_structures_under_sanitizers(sanitized, n, b, gamma, aux):
    res = subprocess.run([sanitized["nd_emulation"], str(n), str(b), str(gamma), str(aux)],
                         capture_output=True, text=True, env=ENV, timeout=600)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert float(res.stdout.strip().splitlines()[-1].split()[-1]) < 1e-10
