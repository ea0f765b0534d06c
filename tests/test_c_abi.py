"""The C ABI from a plain C program (tests/c_abi_smoke.c) that links only
libptsg.so: it compiles and links on the CPU; on a GPU it runs one sample
through steps, swaps, a measurement and a checkpoint, and checks unit
spins, the energies against Eq. (1) evaluated in C, the permutations and an
exact resume."""
import os
import subprocess

import pytest

from paper_1309_1599_amd import ptsg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1309_1599_amd")


def _build(tmp_path):
    if not os.path.exists(ptsg.LIB_PATH):
        from paper_1309_1599_amd import build
        build.build()
    exe = str(tmp_path / "c_abi_smoke")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Werror", f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "c_abi_smoke.c"), "-o", exe, f"-L{PKG}", "-lptsg", "-lm",
           "-Wl,-rpath-link,/opt/rocm/lib", f"-Wl,-rpath,{PKG}:/opt/rocm/lib"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_c_program_compiles_and_links(tmp_path):
    assert os.access(_build(tmp_path), os.X_OK)


@pytest.mark.gpu
def test_c_program_runs(tmp_path):
    exe = _build(tmp_path)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stderr
