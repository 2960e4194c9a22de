"""CPU check of the nested-dissection host structures (Section 4.1): the
elimination tree, the front column lists and child maps, the padding of the
fronts and the use of K = F_II^-1 F_IB in both passes.  tests/nd_emulation.cpp
factors and solves every auxiliary problem of a host-only 3D plan on the CPU
(complex double), organised exactly as the device path, and checks each
solution's residual against the slab operator written out independently."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIBDIR = os.path.join(ROOT, "paper_1504_04058_amd")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    if not os.path.exists(os.path.join(LIBDIR, "libasp.so")):
        pytest.fail("libasp.so is not built")
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("nd") / "nd_emulation")
    cmd = [hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", os.path.join(HERE, "nd_emulation.cpp"), "-o", exe,
           "-I" + os.path.join(LIBDIR, "csrc"), "-I" + os.path.join(ROOT, "include"),
           "-L" + LIBDIR, "-lasp", "-Wl,-rpath," + LIBDIR]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return exe


@pytest.mark.parametrize("n,b,gamma,aux", [(9, 3, 2, 0), (11, 3, 3, 0), (14, 2, 3, 2), (17, 4, 4, 3)])
def test_multifrontal_structures_solve_each_slab(emulator, n, b, gamma, aux):
    res = subprocess.run([emulator, str(n), str(b), str(gamma), str(aux)], capture_output=True,
                         text=True, timeout=600)
    assert res.returncode == 0, res.stdout[-3000:] + res.stderr[-1000:]
    worst = float(res.stdout.strip().splitlines()[-1].split()[-1])
    assert worst < 1e-10
